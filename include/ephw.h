/*
 * ephw.h - C ABI of libephw, Wannier-to-Bloch interpolation of electron-phonon
 * matrix elements on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates Eq. (7) of arXiv:2603.10295,
 *
 *   g_{mn nu}(k,q) = sum_{m'n' kappa alpha} sum_{Re,Rp} g_{m'n' kappa alpha}(Re,Rp)
 *                    U_{mm'}(k+q) U*_{nn'}(k) u_{kappa alpha, nu}(q) e^{i(q.Rp + k.Re)},
 *
 * through the nested loop of Eqs. (9)-(10): per batch of q points the Rp phase
 * sum (Eq. (9)) is one complex GEMM, the mode vectors u(q) are applied once per
 * q, the Re phase sum (Eq. (10)) is one complex GEMM over all k, and the band
 * rotations are applied per (k, q) pair.  U(k) and u(q) come from Hermitian
 * eigensolves of the interpolated H(k) and D(q), done on the GPU in FP64.
 *
 * Conventions
 *   - k, q are fractional coordinates (reciprocal-lattice units); lattice
 *     vectors R are integer triples.  Every phase is w_R * exp(+2 pi i p.R)
 *     with the argument p.R reduced to (-1/2, 1/2] in FP64 before the sine and
 *     cosine; w_R are optional Wigner-Seitz degeneracy weights (NULL = 1).
 *   - H(k) = sum_R w_R e^{2 pi i k.R} H(R), H(R)_{ab} = <w_a(0)|H|w_b(R)>.  Its
 *     eigenvector columns V(k) fix the gauge of Eq. (5) as U(k) = V(k)^dagger,
 *     so the band factors of Eq. (7) are V(k+q)^dagger g V(k).
 *   - D(q) = sum_R w_R e^{2 pi i q.R} C(R) / sqrt(M_kappa M_kappa');
 *     u_{kappa alpha, nu}(q) = e_{kappa alpha, nu}(q) / sqrt(M_kappa) (mode
 *     index kappa alpha = 3 kappa + alpha); omega = sqrt(|lambda|).
 *   - Eigenvalues are ascending; each eigenvector column is scaled so that its
 *     largest-magnitude component is real and positive.
 *
 * Memory
 *   - ephw_system_load copies the Wannier-space tensors from HOST memory into
 *     library-owned device memory, where they stay until ephw_system_free (the
 *     e-ph matrix g(Re,Rp) is uploaded once and reused for every k and q).
 *   - Every other pointer argument is DEVICE memory owned by the caller
 *     (k/q lists, index tables, outputs).  The library keeps no pointer to
 *     caller memory after a call returns.
 *   - Complex numbers are interleaved (re, im) pairs: "c128" is two doubles,
 *     "c64" two floats.  All arrays are dense row-major in the index order
 *     given at each argument.
 *
 * Streams and errors
 *   - Compute calls take `stream` (a hipStream_t; NULL = the null stream),
 *     enqueue their work on it and return; the caller synchronises.
 *   - Every function returns an ephw_status.  Argument errors are detected on
 *     the host before anything is enqueued (EPHW_EINVAL, EPHW_EUNSUPPORTED);
 *     ephw_last_error() gives a description (thread-local).  Errors raised by
 *     kernels (an eigensolve that did not converge, an out-of-range index in a
 *     k+q table) are recorded in a device status word of the context and read
 *     by ephw_ctx_check().
 *   - Calls that share a system or k-set use that object's workspace and must
 *     be issued on one stream (or be externally ordered).
 */
#ifndef EPHW_H
#define EPHW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ephw_status;
#define EPHW_OK            0
#define EPHW_EINVAL        1  /* invalid argument (shape, NULL pointer, range) */
#define EPHW_ENOMEM        2  /* device allocation failed */
#define EPHW_EDEVICE       3  /* HIP runtime error */
#define EPHW_ENOCONV       4  /* a Jacobi eigensolve hit its sweep limit */
#define EPHW_EUNSUPPORTED  5  /* a valid request the library does not handle */
#define EPHW_EINDEX        6  /* a k+q index table entry was out of range */

/* arithmetic of the phase sums and rotations; eigensolves are always FP64 */
#define EPHW_FP64        0  /* complex128 GEMMs on FP64 MFMA, g stored c128 */
#define EPHW_FP32        1  /* complex64 GEMMs on FP32 MFMA, g stored c64 */
#define EPHW_FP32_COMP   2  /* compensated FP32: as EPHW_FP32, but each phase sum
                               accumulates in K blocks of 32 (fresh FP32 MFMA
                               accumulators per block, block sums added in FP32),
                               which cuts the FP32 accumulation error, the
                               dominant one, about 3x; backward, Eq. (6) and
                               batches take FP64 or FP32 sets only */

/* storage type of g(Re,Rp) */
#define EPHW_C128 0
#define EPHW_C64  1

/* output selection for ephw_interpolate (bit flags) */
#define EPHW_OUT_G          1u  /* store g_{mn nu}(k,q) */
#define EPHW_OUT_BAND_SUM   2u  /* store T_nu(k,q) = sum_mn |g_{mn nu}|^2 (gauge free) */
#define EPHW_OUT_LOSS       4u  /* accumulate L += sum w_{mn nu}(k,q) |g_{mn nu}|^2 */
#define EPHW_OUT_WANNIER    8u  /* skip the band and mode rotations: store the
                                   Re/Rp phase sums g_{m'n' kappa alpha}(k,q) */

/* grouping of a (k, q) pair list (ephw_window_pairs, ephw_interpolate_pairs) */
#define EPHW_PAIRS_BY_Q   0  /* CSR over the q list; the other index of a pair is k */
#define EPHW_PAIRS_BY_K   1  /* CSR over the k-set; the other index of a pair is q */
#define EPHW_PAIRS_AUTO  -1  /* ephw_window_pairs picks the cheaper of the two */

typedef struct ephw_ctx ephw_ctx;
typedef struct ephw_system ephw_system;
typedef struct ephw_kset ephw_kset;

/* Create a context on HIP device `device`.  Allocates the device status word. */
ephw_status ephw_ctx_create(int device, ephw_ctx** out);
ephw_status ephw_ctx_destroy(ephw_ctx* ctx);

/* Synchronise `stream`, read and clear the context's device status word.
   Returns EPHW_OK, EPHW_ENOCONV or EPHW_EINDEX. */
ephw_status ephw_ctx_check(ephw_ctx* ctx, void* stream);

/* Limits of a context (blocking; waits for the device to go idle).
     max_device_bytes  cap on the device memory held by the context's systems,
                       k-sets and batches (tensors, workspaces, caches); an
                       allocation that would pass it fails with EPHW_ENOMEM
                       before any device allocation is attempted.  0 = no cap.
     max_sweeps        Jacobi sweeps an eigensolve may take before it stops and
                       raises EPHW_ENOCONV in the status word (the kernel still
                       writes its current eigenvalues and vectors and exits
                       normally); 0 <= max_sweeps <= 1000, default 40 (an order-n
                       solve converges in well under 20 for n <= 256). */
ephw_status ephw_ctx_set_limits(ephw_ctx* ctx, int64_t max_device_bytes, int32_t max_sweeps);
/* device memory the context's objects hold now, and its cap (0 = none) */
ephw_status ephw_ctx_memory(const ephw_ctx* ctx, int64_t* used, int64_t* limit);

/* Wannier-space description of one material (Eqs. (3)-(5) inputs).  All
   pointers are HOST memory.  nm = 3*na.
     r_e [ne][3], r_p [np][3], r_h [nh][3], r_c [nc][3]   int32 lattice vectors
     w_e [ne], w_p [np], w_h [nh], w_c [nc]               f64 weights or NULL (= 1)
     h_r  [nh][nw][nw]            c128, H(R)
     c_r  [nc][nm][nm]            f64, force constants C(R) (real)
     mass [na]                    f64, atomic masses (> 0)
     g    [np][ne][nm][nw][nw]    e-ph matrix g_{m'n' kappa alpha}(Re,Rp) of
                                  Eq. (3), element type given by g_dtype      */
typedef struct ephw_system_desc {
  int32_t nw, na;
  int64_t ne, np, nh, nc;
  const int32_t *r_e, *r_p, *r_h, *r_c;
  const double *w_e, *w_p, *w_h, *w_c;
  const void* h_r;
  const double* c_r;
  const double* mass;
  const void* g;
  int32_t g_dtype;              /* EPHW_C128 or EPHW_C64 */
} ephw_system_desc;

/* Copy a system to the device (blocking).  Limits: 1 <= nw <= 256,
   1 <= na <= 86 (nm <= 258), every n >= 1.  g may be NULL: its device copy
   is then allocated but not written, and must be filled with
   ephw_system_set_g before any call reads it (for g generated on the
   device, e.g. systems too large to stage on the host). */
ephw_status ephw_system_load(ephw_ctx* ctx, const ephw_system_desc* desc, ephw_system** out);
ephw_status ephw_system_free(ephw_system* sys);
/* Replace the system's g(Re,Rp) by `g` (DEVICE memory, same shape and element
   type as at load), copied on `stream`; k-sets of the system stay valid. */
ephw_status ephw_system_set_g(ephw_system* sys, const void* g, void* stream);
/* Release the system's workspaces (the buffers its calls grow and keep for
   reuse; the next call allocates them again).  Waits for the device. */
ephw_status ephw_system_trim(ephw_system* sys);
/* bytes of library-owned device memory held by the system (tensors + workspace) */
ephw_status ephw_system_bytes(const ephw_system* sys, int64_t* bytes);

/* Electron bands on a k list (H(k) interpolation + FP64 eigensolve): the
   gauge matrices of Eq. (5) (U(k) = V(k)^dagger; Results, "Computational
   aspects of electron-phonon matrix interpolation") and the band energies the
   energy window and the downstream reductions use.
     k    [nk][3] f64 (device)
     eps  [nk][nw] f64 (device) or NULL
     vecs [nk][nw][nw] c128 (device) or NULL; column j is the eigenvector of eps[j]
   vecs must be 16-byte aligned, as every c128 array is (EPHW_EINVAL otherwise). */
ephw_status ephw_bands(ephw_system* sys, const double* k, int64_t nk, double* eps, void* vecs,
                       void* stream);

/* Phonons on a q list (D(q) interpolation + FP64 eigensolve): the mode
   vectors u(q) that Eq. (2) projects the perturbing potential on, and the
   frequencies omega(q).
     q     [nq][3] f64 (device)
     lam   [nq][nm] f64 eigenvalues of D(q), or NULL
     omega [nq][nm] f64 sqrt(|lam|), or NULL
     evecs [nq][nm][nm] c128 eigenvectors e (columns), or NULL  (u = e/sqrt(M)),
           16-byte aligned (EPHW_EINVAL otherwise) */
ephw_status ephw_phonons(ephw_system* sys, const double* q, int64_t nq, double* lam,
                         double* omega, void* evecs, void* stream);

/* Eq. (9) alone: g(Re,q) = sum_Rp w_Rp e^{2 pi i q.Rp} g(Re,Rp).
     q   [nq][3] f64 (device)
     out [nq][ne][nm][nw][nw] c128 (EPHW_FP64) or c64 (EPHW_FP32*) (device)
   The precision must match the stored g (FP64 <-> c128, FP32 <-> c64). */
ephw_status ephw_phase_sum_rp(ephw_system* sys, const double* q, int64_t nq, int32_t prec,
                              void* out, void* stream);

/* A prepared set of fine k points: their phases e^{2 pi i k.Re}, bands eps(k)
   and eigenvectors V(k), kept on the device and reused by every
   ephw_interpolate call on that set (the k loop of Eq. (10)).
     k [nk][3] f64 (device), copied. */
ephw_status ephw_kset_create(ephw_system* sys, const double* k, int64_t nk, int32_t prec,
                             void* stream, ephw_kset** out);
ephw_status ephw_kset_free(ephw_kset* ks);
/* copy eps(k) [nk][nw] f64 and/or V(k) [nk][nw][nw] c128 (device) out of the set */
ephw_status ephw_kset_bands(ephw_kset* ks, double* eps, void* vecs, void* stream);

/* Eq. (7) on every pair of the k-set's points with the q list.
     q        [nq][3] f64 (device)
     kq_index [nq][nk] int32 (device) or NULL.  If given, V(k_i + q_j) is taken as
              V(k_{kq_index[j][i]}) of the k-set (k+q on the k grid); otherwise
              H(k+q) is interpolated and diagonalised for every pair.
     q_offset index of q[0] in the caller's full q list (enters the loss weights)
     prec     EPHW_FP64 / EPHW_FP32 / EPHW_FP32_COMP; must match the k-set's
     flags    EPHW_OUT_* bits
     g_out    [nq][nk][nm][nw][nw] c128 (FP64) or c64 (FP32*), if EPHW_OUT_G;
              with EPHW_OUT_WANNIER the same shape holds the unrotated sums
              (index order [q][k][kappa alpha][m'][n'])
     band_sum [nq][nk][nm] f64, if EPHW_OUT_BAND_SUM
     loss     one f64, if EPHW_OUT_LOSS: L += sum w |g|^2 with
              w = 0.5 + (x >> 40) 2^-24, x the i-th SplitMix64 output for seed
              loss_seed and i = ((((q_offset+iq)*nk + ik)*nm + nu)*nw + m)*nw + n
     eps_kq   [nq][nk][nw] f64 or NULL: bands at k+q
     omega    [nq][nm] f64 or NULL
   Returns EPHW_EINVAL for inconsistent arguments before enqueuing anything. */
ephw_status ephw_interpolate(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                             int64_t q_offset, int32_t prec, uint32_t flags, void* g_out,
                             double* band_sum, double* loss, uint64_t loss_seed, double* eps_kq,
                             double* omega, void* stream);

/* ephw_interpolate for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   same arguments, outputs and results, but every intermediate buffer (phase
   factors, mode vectors, the g(Re,q) sweeps, the Re-sum output, loss
   partials, k+q eigensolves) lives in a static scratch array of the library,
   256 MiB per device, which each device the library runs on holds until the
   process ends.  No device memory is allocated or freed by the call.
   - The q points are processed in batches small enough for the scratch (at
     most the batch ephw_interpolate would take).  A call whose buffers do not
     fit even at one q per batch returns EPHW_ENOMEM before enqueuing anything
     (the per-call part grows with nq: split long q lists over calls).
   - Every call on a device shares that device's scratch and leaves its
     contents behind: calls that overlap on one device (different streams,
     threads or processes sharing a context's device) race and must be
     ordered by the caller.  Nothing in the scratch needs to start at zero.
   - Systems with more than 32 bands return EPHW_EUNSUPPORTED.
   - No stage events are recorded (ephw_profile_* does not see these calls). */
ephw_status ephw_interpolate_noalloc(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                     int64_t q_offset, int32_t prec, uint32_t flags, void* g_out,
                                     double* band_sum, double* loss, uint64_t loss_seed, double* eps_kq,
                                     double* omega, void* stream);

/* Eq. (6): the coarse Bloch -> Wannier transform, the inverse of Eq. (7)
   when the k-set and the q list are the coarse grids commensurate with the
   Re and Rp sets (complete residue boxes, k'+q' on the k grid):
     g(Re,Rp) = 1/(Ne Np) sum_{k',q'} e^{-2 pi i (k'.Re + q'.Rp)}
                sum_nu [V(k'+q') g_nu(k',q') V(k')^dagger] u^-1_{nu,ka}(q')
   with U = V^dagger as in Eq. (7), u = e/sqrt(M) the mode vectors of D(q'),
   and no lattice-vector weights (Eq. (6) has none).
     ks       k-set on the coarse k' grid (its eigenvectors are V(k'))
     q        [nq][3] f64 (device): the coarse q' points, nq >= 1
     kq_index [nq][nk] int32 (device), required: grid index of k'_i + q'_j in the set
     g_bloch  [nq][nk][nm][nw][nw] (device): c128 for an FP64 set, c64 for FP32,
              in the layout ephw_interpolate stores
     g_out    [np][ne][nm][nw][nw] (device), same element type, overwritten
   EPHW_FP32_COMP sets are not supported.  Enqueued on stream. */
ephw_status ephw_wannier_transform(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                   const void* g_bloch, void* g_out, void* stream);

/* Energy-window prescreening (the Results section's single-node benchmark
   skips the matrix elements of states outside an energy window before
   interpolating; its practical guidance notes that the window cuts both the
   contributing k points and bands).  A k point of the set is
   active when one of its bands lies in [e_lo, e_hi], a pair (k, q) when k
   and k+q both are, and a q point when it has an active pair.  Outputs, for
   running Eq. (7) on the active points only (a k-set made from k_out, the q
   list q_out, the index table kq_out):
     k_out     [nk][3] f64 (device): the active k points, ascending set order,
               in the first *nk_out rows
     nk_out    host int64: number of active k points
     q_out     [nq][3] f64 (device): the active q points (first *nq_out rows)
     nq_out    host int64
     kq_out    [nq][nk] int32 (device): its first nq_out*nk_out entries, row
               r = active q, column c = active k, hold the position of k+q in
               k_out, or 0 where k+q is outside the window
     pair_mask [nq][nk] uint8 (device) or NULL: same layout, 1 where k+q is in
               the window (those pairs are the ones to keep)
   kq_index [nq][nk] int32 (device, required for nq > 0): grid index of k+q
   in the set; entries outside [0, nk) count as inactive and set the
   context's status word (EPHW_EINDEX from ephw_ctx_check).  The call
   synchronises the stream (the counts are host values). */
ephw_status ephw_window_screen(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index, double e_lo,
                               double e_hi, double* k_out, int64_t* nk_out, double* q_out, int64_t* nq_out,
                               int32_t* kq_out, uint8_t* pair_mask, void* stream);

/* The kept pairs of the same energy window as a list (the pre-screening of
   the Results section's single-node benchmark, taken down to single (k, q)
   pairs): pair (k, q) is kept when k and k+q (kq_index) both have a band in
   [e_lo, e_hi].  The list is grouped (CSR) by q or by k:
     order      EPHW_PAIRS_BY_Q, EPHW_PAIRS_BY_K, or EPHW_PAIRS_AUTO: by k when
                fewer k than q own a kept pair (the cheaper nesting order for
                ephw_interpolate_pairs), else by q
     order_out  host int32 or NULL: the grouping used
     pair_start HOST int64, [nq + 1] (by q) or [nk + 1] (by k; for AUTO give
                max(nq, nk) + 1): the pairs of group j are
                p = pair_start[j] .. pair_start[j+1]-1; the last entry is the total
     pair_other [capacity] int32 (device): k index in the set (by q) or q index
                in the list (by k) of pair p, ascending within each group
     pair_kq    [capacity] int32 (device): kq_index[q][k] of pair p, the set
                index of k+q
     band_range host int32 [2] or NULL: the first band and the number of
                bands of the smallest band range that holds every band with
                an energy in the window at some k of the set (the band window
                of ephw_interpolate_pairs; 0, 0 when no band is in the window)
   kq_index [nq][nk] int32 (device): as in ephw_window_screen (entries outside
   [0, nk) count as dropped and set EPHW_EINDEX in the status word).
   pair_start is always written; when the total exceeds `capacity` the call
   returns EPHW_EINVAL without writing the device lists (the caller can size
   them from the total and call again).  Synchronises the stream. */
ephw_status ephw_window_pairs(ephw_kset* ks, const int32_t* kq_index, int64_t nq, double e_lo, double e_hi,
                              int32_t order, int32_t* order_out, int64_t* pair_start, int32_t* pair_other,
                              int32_t* pair_kq, int64_t capacity, int32_t* band_range, void* stream);

/* Eq. (7) on a list of (k, q) pairs (Nw <= 32; FP64 or FP32 k-sets) in the
   form ephw_window_pairs writes (order EPHW_PAIRS_BY_Q or EPHW_PAIRS_BY_K;
   pair_start HOST; pair_other and pair_kq device [pair_start[last]]): for
   pair p, with k = its k-set index and q = its row of the list q [nq][3] f64
   (device), computes the g_{mn nu}(k, q) that ephw_interpolate gives at that
   k and q with the k+q grid index pair_kq[p].  Only kept pairs enter the
   phase sums' pair stage and the rotations.  The grouping selects the
   nesting order of the two phase sums:
     by q: per q, Eq. (9) over all Re (one GEMM per batch of q), then the Re
           sum of Eq. (10) for that q's kept k only;
     by k: per k, the Re sum first over all Rp (one batched GEMM per chunk of
           k), then the Rp sum of Eq. (9) for that k's kept q only, then the
           mode vectors u(q) per pair.
   The first stage costs (points of its group that own a pair) x Ne x Np x
   Nw^2 Nm, the second (kept pairs) x (Ne or Np) x Nw^2 Nm, so grouping by
   the index with fewer such points is the cheaper order.
     flags, loss_seed, q_offset  as in ephw_interpolate; the loss weights use
              the element index of (q_offset + q, k) in the k-set, so the loss
              equals that of ephw_interpolate over the same pairs
     band_lo, band_count  band window (the window's practical effect on the
              bands): band_count > 0 keeps bands band_lo .. band_lo+band_count-1
              at k+q (m) and at k (n) only: the rotations form just those rows
              and columns, and g, the band sums and the loss cover just those
              elements (loss weights keep their full-layout indices);
              band_count = 0 keeps all Nw bands.  Not with EPHW_OUT_WANNIER.
     g_out    [npairs][nm][nb][nb] c128 (FP64) or c64 (FP32), nb = band_count
              or Nw, if EPHW_OUT_G
     band_sum [npairs][nm] f64, if EPHW_OUT_BAND_SUM
     loss     one f64 (L +=), if EPHW_OUT_LOSS
   pair_start must start at 0 and not decrease (checked on the host); pair
   indices outside the k-set or the q list set EPHW_EINDEX in the status
   word.  The call copies its group offsets and per-group GEMM descriptors to
   the device through pinned host memory the system owns; it does not
   synchronise the stream. */
ephw_status ephw_interpolate_pairs(ephw_kset* ks, const double* q, int64_t nq, int32_t order,
                                   const int64_t* pair_start, const int32_t* pair_other, const int32_t* pair_kq,
                                   int64_t q_offset, int32_t prec, uint32_t flags, int32_t band_lo,
                                   int32_t band_count, void* g_out, double* band_sum, double* loss,
                                   uint64_t loss_seed, void* stream);

/* A downstream reduction of stored matrix elements over q (the multi-node
   scalability runs of the Results section compute an electron self-energy
   of MoS2 from the interpolated g; the formula is not printed there): the
   phonon-limited linewidth, the imaginary part of the Fan-Migdal self-energy
   with Gaussian broadening,
     gamma[k][n] += pi / nq_total * sum over q, modes nu with omega >= omega_min, bands m of
        |g_{mn nu}(k,q)|^2 / (2 omega) * [ (N + f_m) G(e_n - e_m + omega) + (N + 1 - f_m) G(e_n - e_m - omega) ]
   with e_n = eps_k[k][n], e_m = eps_kq[q][k][m], omega = omega[q][nu],
   N = 1/(exp(omega/T) - 1), f_m = 1/(exp((e_m - mu)/T) + 1) and
   G(x) = exp(-x^2 / (2 sigma^2)) / (sigma sqrt(2 pi)).  The 1/(2 omega) is the
   zero-point amplitude that the mode vectors e/sqrt(M) of Eq. (2) leave out.
   Calls on successive q chunks accumulate; nq_total is the full q count.
     prec    EPHW_FP64: g c128; EPHW_FP32 / EPHW_FP32_COMP: g c64
     g       [nq][nk][nm][nw][nw] (device), as ephw_interpolate stores it
     eps_k [nk][nw], eps_kq [nq][nk][nw], omega [nq][nm]: f64 (device)
     gamma   [nk][nw] f64 (device), accumulated (+=), caller-owned
   temperature, sigma > 0 (energy units of eps); omega_min >= 0 drops soft modes,
   and modes with omega = 0 never contribute (1/(2 omega) is undefined there).
   Callers should pass omega_min > 0: acoustic modes near q = 0, and modes of an
   unstable D(q) (lambda < 0, omega = sqrt(|lambda|)), have small nonzero omega
   whose weight ~ T / omega^2 would dominate gamma.
   Occupations and sums are FP64; the Gaussians are FP32 for c64 g.
   Deterministic: every sum runs in a fixed order. */
ephw_status ephw_linewidth(int32_t prec, const void* g, int64_t nq, int64_t nk, int32_t nm, int32_t nw,
                           const double* eps_k, const double* eps_kq, const double* omega, double temperature,
                           double mu, double sigma, double omega_min, int64_t nq_total, double* gamma,
                           void* stream);

/* The reduction of ephw_linewidth applied to Eq. (7)'s matrix elements as they
   are formed, without storing them (the way the paper's self-energy runs
   consume g): gamma[k][n] += the sum over this q list, with the weights, the
   1/(2 omega) amplitude and the parameters of ephw_linewidth, of
   |g_{mn nu}(k,q)|^2 for every point k of the set.  eps_k, eps_kq and omega are
   the library's own (the k-set's bands, the bands at k+q, sqrt(|lambda(q)|)).
   For FP32 k-sets with Nw of 4 or 8 the rotations and the reduction run in the
   epilogue of the Eq. (10) GEMM; otherwise each q batch's g goes through a
   library workspace and the ephw_linewidth kernel.  Per-batch sums are added
   in a fixed order (deterministic).
     kq_index  [nq][nk] int32 or NULL, as in ephw_interpolate
     gamma     [nk][nw] f64 (device), accumulated (+=)
   Systems with more than 32 bands return EPHW_EUNSUPPORTED. */
ephw_status ephw_interpolate_linewidth(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                       double temperature, double mu, double sigma, double omega_min,
                                       int64_t nq_total, double* gamma, void* stream);

/* Gauge-invariant |g|^2 of stored matrix elements (the quantity Eq. (7)'s
   results are compared by: eigenvectors of (near-)degenerate eigenvalues are
   fixed only up to a unitary mixing inside their block).  For every pair,
   element (nu, m, n) of out is the sum of |g_{m'n'nu'}|^2 over nu' in the
   block of nu (modes at q), m' in the block of m (bands at k+q) and n' in the
   block of n (bands at k), so every element of a block holds the block's sum.
   A block is a run of the ascending list whose consecutive gaps are at most
   rel_tol * max(1, max |value|) of that list (1e-6 is the usual choice).
     prec    EPHW_FP64: g c128; EPHW_FP32 or EPHW_FP32_COMP: g c64
     g       [nq][nk][nm][nw][nw] (device), as ephw_interpolate stores it
     eps_kq  [nq][nk][nw] f64 (device), ascending: bands at k+q
     eps_k   [nk][nw] f64 (device), ascending: bands at k
     lam     [nq][nm] f64 (device), ascending: eigenvalues of D(q) (ephw_phonons)
     out     [nq][nk][nm][nw][nw] f64 (device), caller-owned
   Limits: 1 <= nw <= 256, 1 <= nm <= 258.  Enqueued on stream. */
ephw_status ephw_degenerate_sums(int32_t prec, const void* g, int64_t nq, int64_t nk, int32_t nm, int32_t nw,
                                 const double* eps_kq, const double* eps_k, const double* lam, double rel_tol,
                                 double* out, void* stream);

/* Loss and gradients (not in the paper: the adjoint of Eq. (7)).
   L = sum over the k-set's points and the q list of w_{mn nu}(k,q) |g_{mn nu}(k,q)|^2
   with the SplitMix64 weights of EPHW_OUT_LOSS (seed loss_seed, q index q_offset + iq).
   One call recomputes the forward in (q batch, k tile) units and accumulates
     loss   one f64: L +=
     dL_dg  [np][ne][nm][nw][nw] c128 (FP64 k-set) or c64 (FP32), +=, gradient
            dL/dRe g + i dL/dIm g with respect to the stored g(Re,Rp)
     dL_dk  [nk][3] f64 +=, gradient with respect to the fractional k coordinates
     dL_dq  [nq][3] f64 +=
   (any of them may be NULL).  kq_index [nq][nk] (k+q on the k grid) is
   required; V(k+q) is the k-set's eigenvector at that grid point, and its
   derivative there gives both dL/dk and dL/dq of the pair.  Eigenvectors enter
   through their first-order change dV = V (F o (V^dagger dH V)),
   F_ij = 1/(eps_j - eps_i) (non-degenerate spectra). */
ephw_status ephw_loss_backward(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                               int64_t q_offset, uint64_t loss_seed, double* loss, void* dL_dg,
                               double* dL_dk, double* dL_dq, void* stream);

/* Tuning knobs (0 = automatic).  q_batch: q points per Rp/Re GEMM sweep. */
ephw_status ephw_set_q_batch(ephw_system* sys, int32_t q_batch);
/* k points per tile of the unit loops (large-band rotations, the adjoint) */
ephw_status ephw_set_k_tile(ephw_system* sys, int32_t k_tile);

/* Per-stage GPU timing for benchmarks: while enabled, every stage of the calls
   made on `sys` (and its k-sets) is bracketed by HIP events recorded on the
   call's stream.  ephw_profile_read synchronises those events, writes the
   summed milliseconds and launch counts of each stage (arrays of
   EPHW_NSTAGES entries; either may be NULL) and clears the records. */
#define EPHW_STAGE_PHASE     0  /* phase factors */
#define EPHW_STAGE_EIG       1  /* H(k), D(q) interpolation + eigensolve */
#define EPHW_STAGE_KQ_EIG    2  /* H(k+q) interpolation + eigensolve per pair */
#define EPHW_STAGE_RP_GEMM   3  /* Eq. (9) phase sum */
#define EPHW_STAGE_MODE_ROT  4  /* u(q) applied to g(Re,q) */
#define EPHW_STAGE_RE_GEMM   5  /* Eq. (10) Re phase sum */
#define EPHW_STAGE_BAND_ROT  6  /* V(k+q)^dagger g V(k) + epilogues */
#define EPHW_STAGE_OTHER     7  /* casts, gathers, reductions */
#define EPHW_NSTAGES         8
ephw_status ephw_profile_enable(ephw_system* sys, int32_t enable);
ephw_status ephw_profile_read(ephw_system* sys, double* ms, int64_t* launches);

/* ---------------------------------------------------------------------------
   Many systems in one pass (not in the paper: persistent multi-system batching).
   Each item interpolates one k-set (of its own system) with a q list whose
   k+q fall on the k grid (kq_index is required).  Per item, a shape (q points
   per sweep, k points per tile, GEMM tile configuration) is chosen by the
   autotuner; the pass then runs in rounds, and every stage of a round (the
   Eq. (9) GEMMs, mode rotations, Eq. (10) GEMMs, band rotations, loss sums)
   is one grouped launch over all systems; the GEMM stages are persistent
   launches striding over the tiles of every system.  The whole pass is
   captured once into a HIP graph and replayed by ephw_batch_run.
   Outputs are the pointers given at ephw_batch_create (fixed for the batch's
   lifetime); loss outputs accumulate (L +=) on every run.
   --------------------------------------------------------------------------- */
typedef struct ephw_batch ephw_batch;
typedef struct ephw_batch_item {
  ephw_kset* ks;             /* k set; its system and precision are used */
  const double* q;           /* [nq][3] f64 (device) */
  int64_t nq;
  const int32_t* kq_index;   /* [nq][nk] int32 (device), required */
  uint32_t flags;            /* EPHW_OUT_G / EPHW_OUT_BAND_SUM / EPHW_OUT_LOSS */
  void* g_out;               /* as in ephw_interpolate */
  double* band_sum;
  double* loss;
  uint64_t loss_seed;
} ephw_batch_item;
typedef struct ephw_batch_options {
  int32_t tune;              /* 0: heuristic shapes; 1: time candidate shapes on the device */
  const char* tune_cache;    /* file of tuned shapes (one JSON object per line) or NULL */
  int32_t use_graph;         /* 1: capture the pass into a HIP graph */
  int64_t item_workspace_bytes; /* per-item cap of the sweep buffers; 0: what the
                                   item's largest unit (128 q, every k) needs, between
                                   1 GiB and 8 GiB, within workspace_budget_bytes (below) */
  int64_t workspace_budget_bytes; /* with item_workspace_bytes = 0: device memory the
                                   sweep buffers may take together; 0: half of the free
                                   device memory.  When the items' caps add up to more,
                                   the largest items run solo (their rounds after the
                                   grouped ones, one item at a time, sharing one sweep
                                   region) until the rest fit beside that region; the
                                   remaining caps are scaled down only if even that
                                   does not fit.  A solo item's phase sums run as plain
                                   GEMMs of its own shape, so its results can differ from
                                   the grouped form's by rounding only.  (Field added in
                                   version 0.2.0.) */
} ephw_batch_options;
/* Plan a batch: validates items, tunes shapes, allocates the workspace.
   All items must share one precision; nw <= 32 and nm <= 24 per system. */
ephw_status ephw_batch_create(ephw_ctx* ctx, const ephw_batch_item* items, int32_t n,
                              const ephw_batch_options* opt, void* stream, ephw_batch** out);
ephw_status ephw_batch_run(ephw_batch* b, void* stream);
/* the shape chosen for item i: q points per sweep, k points per tile, GEMM tile
   configuration of the Eq. (9) and Eq. (10) GEMMs (0 = 128-row tiles, 1 = 64x64) */
ephw_status ephw_batch_shape(const ephw_batch* b, int32_t i, int32_t* q_batch, int32_t* k_tile,
                             int32_t* cfg_rp, int32_t* cfg_re);
/* number of rounds and of kernel launches in one pass */
ephw_status ephw_batch_stats(const ephw_batch* b, int32_t* rounds, int32_t* launches);
/* *solo = 1 if item i runs its rounds on its own (see workspace_budget_bytes), else 0;
   EPHW_EINVAL for a NULL batch or output, or no such item.  (Since version 0.2.0.) */
ephw_status ephw_batch_solo(const ephw_batch* b, int32_t i, int32_t* solo);
ephw_status ephw_batch_free(ephw_batch* b);

const char* ephw_status_string(ephw_status s);
const char* ephw_last_error(void);
/* library version as MAJOR*10000 + MINOR*100 + PATCH */
int32_t ephw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EPHW_H */
