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
// the LDS sized to the order (8 KB at n = 11) so that a CU holds as many
// solves as its registers allow; each lane owns one 2x2 block of the round
// (below).  Large matrices (n > 32) live in a global workspace, one 1024-thread
// workgroup per matrix (the rotation parameters stay in LDS).
#include "kernels.h"

namespace ephw {
namespace {

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
                            double* rs, double* rer, double* rei, int* rp, int* rq, double* red, int max_sweeps) {
  const int tid = threadIdx.x;
  const int n2 = n + (n & 1);
  const int npairs = n2 / 2;
  for (int e = tid; e < n * n; e += NT) {
    Vr[e] = (e / n == e % n) ? 1.0 : 0.0;
    Vi[e] = 0.0;
  }
  __syncthreads();
  bool converged = (n <= 1);
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
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
constexpr int kSmallPerBlock = 4;  // small solves (wavefronts) per workgroup

// ---------------------------------------------------------------------------
// Small solves (n <= 32): one 64-lane wavefront per matrix, A and V in LDS as
// interleaved complex with the order padded to N2 = 2 NP (a zero row and
// column for odd n, whose pair is then the identity).  In each round of the
// tournament the NP disjoint planes cut A and V into NP^2 2x2 blocks, rows
// {p_i, q_i} x columns {p_j, q_j}.  J_i^H A J_j and V J_j touch only block
// (i, j), so one lane updates a block with no other lane's data.  A stays
// exactly Hermitian: only its upper triangle is kept (an entry below the
// diagonal is read as the conjugate of its transpose) and only blocks with
// i <= j are computed.  The
// NP (NP + 1) / 2 blocks of A and the NP^2 of V are one list of tasks of the
// same shape (V's left rotation is the identity), 57 of them at n = 11, so
// the round is a single pass over the wave.  The sweep's last round sums
// |A|^2 (total and off-diagonal) over the blocks it wrote, so the stopping
// test costs one wave reduction per sweep.
//
// Rotation parameters without divisions, for x = d - a, y = 2|b|:
//   r = sqrt(x^2 + y^2), w = |x| + r, z = 1/sqrt(w^2 + y^2),
//   c = w z, s = sign(x) y z, sigma = s b/|b|,
// which are the t = sign(tau)/(|tau| + sqrt(1 + tau^2)) formulas above with
// the common factors cleared; J = [[c, sigma], [-conj(sigma), c]].
// ---------------------------------------------------------------------------
template <int NP>
struct SmallLayout {
  static constexpr int N2 = 2 * NP;
  static constexpr int NA = NP * (NP + 1) / 2;                   // blocks of A (i <= j)
  static constexpr int NT = NA + NP * NP;                         // tasks: A blocks, then V blocks
  static constexpr int TPL = (NT + 63) / 64;                      // tasks per lane
  static constexpr size_t a_elems = (size_t)N2 * N2;            // complex
  static constexpr size_t prm_elems = 2 * (size_t)NP;            // (c, 0), sigma per pair
  static constexpr size_t fix_elems = (size_t)N2;                // phase fix per column
  static constexpr size_t bytes = (2 * a_elems + prm_elems + fix_elems) * 16 + (size_t)N2 * 4;
  static constexpr size_t slice_elems = (bytes + 15) / 16;       // one wavefront's share, 16-byte units
  // per-round task descriptors and plane pairs, shared by the workgroup's
  // solves (which all have this padded order), when they fit
  static constexpr size_t table_bytes = (size_t)(N2 - 1) * NT * 8 + (size_t)(N2 - 1) * NP * 4;
  static constexpr bool kTable = TPL > 1 && table_bytes <= 32768;
  static constexpr size_t table_elems = kTable ? (table_bytes + 15) / 16 : 0;
};

template <int NP>
__device__ __forceinline__ void decode_task(int t, bool& is_v, int& i, int& j) {
  constexpr int NA = SmallLayout<NP>::NA;
  if (t < NA) {
    int r = 0, rest = t;
    while (rest >= NP - r) {
      rest -= NP - r;
      ++r;
    }
    is_v = false;
    i = r;
    j = r + rest;
  } else {
    const int v = t - NA;
    is_v = true;
    i = v / NP;
    j = v % NP;
  }
}

// plane of pair k in a round: p | q << 8 with p < q
__device__ __forceinline__ int pair_pq(int k, int round, int n2) {
  const int u = player_at(k, round, n2), v = player_at(n2 - 1 - k, round, n2);
  return u < v ? (u | v << 8) : (v | u << 8);
}

// The four entries of task t's block in a round, as offsets into the solve's
// slice (A at 0, V after it); bit 15 marks an entry of A below the diagonal,
// held as the conjugate of its transpose.
template <int NP>
__device__ __forceinline__ uint2 task_entries(int t, int round) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2;
  bool is_v;
  int i, j;
  decode_task<NP>(t, is_v, i, j);
  const int pqi = pair_pq(i, round, N2), pqj = pair_pq(j, round, N2);
  const int rr[2] = {pqi & 0xff, pqi >> 8}, cc[2] = {pqj & 0xff, pqj >> 8};
  uint32_t d[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = rr[e >> 1], c = cc[e & 1];
    d[e] = is_v ? (uint32_t)(L::a_elems + r * N2 + c)
                : (r <= c ? (uint32_t)(r * N2 + c) : (uint32_t)(c * N2 + r) | 0x8000u);
  }
  return make_uint2(d[0] | d[1] << 16, d[2] | d[3] << 16);
}

template <int NP>
__device__ void build_tables(uint2* ent, int* pq) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2;
  for (int e = threadIdx.x; e < (N2 - 1) * L::NT; e += blockDim.x) ent[e] = task_entries<NP>(e % L::NT, e / L::NT);
  for (int e = threadIdx.x; e < (N2 - 1) * NP; e += blockDim.x) pq[e] = pair_pq(e % NP, e / NP, N2);
}

// Position order.  A and V are held with their rows and columns (V: columns)
// in tournament-position order: pair k of every round is positions k and
// N2 - 1 - k, and after each round the indices move to the positions they take
// in the next one.  The move is the same every round (the index at position 1
// goes to the last position, those above 1 move down by one, position 0
// stays), so a lane's block has fixed load addresses and fixed store
// addresses (the moved positions) in every round; after a whole sweep of
// N2 - 1 rounds every index is back at its own position.
__device__ __forceinline__ int next_pos(int pos, int n2) {
  return pos == 0 ? 0 : (pos == 1 ? n2 - 1 : pos - 1);
}

// offset of entry (r, c) of A (upper triangle: an entry below the diagonal is
// the conjugate of its transpose, flagged by bit 15) or of V (after A)
template <int NP>
__device__ __forceinline__ uint32_t entry_offset(bool is_v, int r, int c) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2;
  if (is_v) return (uint32_t)(L::a_elems + r * N2 + c);
  return r <= c ? (uint32_t)(r * N2 + c) : ((uint32_t)(c * N2 + r) | 0x8000u);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// x' = c x - conj(sg) y ; y' = sg x + c y   (one row of [x y] J)
__device__ __forceinline__ void rot_right(double2& x, double2& y, double c, double2 sg) {
  const double2 nx = make_double2(fma(c, x.x, -fma(sg.x, y.x, sg.y * y.y)), fma(c, x.y, -fma(sg.x, y.y, -sg.y * y.x)));
  const double2 ny = make_double2(fma(c, y.x, fma(sg.x, x.x, -sg.y * x.y)), fma(c, y.y, fma(sg.x, x.y, sg.y * x.x)));
  x = nx;
  y = ny;
}

// x' = c x - sg y ; y' = conj(sg) x + c y   (one column of J^H [x; y])
__device__ __forceinline__ void rot_left(double2& x, double2& y, double c, double2 sg) {
  const double2 nx = make_double2(fma(c, x.x, -fma(sg.x, y.x, -sg.y * y.y)), fma(c, x.y, -fma(sg.x, y.y, sg.y * y.x)));
  const double2 ny = make_double2(fma(c, y.x, fma(sg.x, x.x, sg.y * x.y)), fma(c, y.y, fma(sg.x, x.y, -sg.y * x.x)));
  x = nx;
  y = ny;
}

__device__ __forceinline__ double norm2(double2 v) { return v.x * v.x + v.y * v.y; }

// entry descriptor (15-bit offset, conjugate flag in bit 15) -> value
__device__ __forceinline__ double flip_sign(double v, uint32_t d) {
  return __longlong_as_double(__double_as_longlong(v) ^ ((long long)(d & 0x8000u) << 48));
}
__device__ __forceinline__ double2 ld_entry(const double2* X, uint32_t d) {
  const double2 v = X[d & 0x7fffu];
  return make_double2(v.x, flip_sign(v.y, d));
}
__device__ __forceinline__ void st_entry(double2* X, uint32_t d, double2 v) {
  X[d & 0x7fffu] = make_double2(v.x, flip_sign(v.y, d));
}

// the solve of a matrix is one wavefront's (wave_sync, no workgroup barrier)

template <int NP>
__device__ __forceinline__ void jacobi_small_body(const double* __restrict__ H, int n, double* __restrict__ eps,
                                                  double* __restrict__ Vout, uint32_t* status, double tol2, int64_t b,
                                                  double2* slice, int lane, const uint2* ent, const int* pqt) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2;
  double2* A = slice;
  double2* V = A + L::a_elems;
  double2* prm = V + L::a_elems;
  double2* fix = prm + L::prm_elems;
  int* perm = reinterpret_cast<int*>(fix + L::fix_elems);
  const double2* h = reinterpret_cast<const double2*>(H) + b * n * n;
  const double2 zero = make_double2(0.0, 0.0);

  // this lane's tasks, packed as (is_v << 16) | (i << 8) | j; the list does not change between rounds
  int task[L::TPL];
#pragma unroll
  for (int k = 0; k < L::TPL; ++k) {
    const int t = lane + 64 * k;
    int code = -1;
    if (t < L::NT) {
      bool is_v;
      int i, j;
      decode_task<NP>(t, is_v, i, j);
      code = (is_v ? 1 << 16 : 0) | (i << 8) | j;
    }
    task[k] = code;
  }

  double off = 0.0, tot = 0.0;
  for (int e = lane; e < N2 * N2; e += 64) {
    const int r = e / N2, c = e % N2;
    const double2 v = (r < n && c < n) ? h[r * n + c] : zero;
    A[e] = v;
    V[e] = (r == c && r < n) ? make_double2(1.0, 0.0) : zero;
    const double m = norm2(v);
    tot += m;
    off += r != c ? m : 0.0;
  }
  off = wave_sum(off);
  tot = wave_sum(tot);
  wave_sync();
  bool converged = n <= 1 || off <= tol2 * tot;
  off = 0.0;
  tot = 0.0;
  const int max_sweeps = sweep_limit(status);
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
#pragma unroll 1
    for (int round = 0; round < N2 - 1; ++round) {
      if (lane < NP) {
        const int pq = L::kTable ? pqt[round * NP + lane] : pair_pq(lane, round, N2);
        const int p = pq & 0xff, q = pq >> 8;
        double c = 1.0;
        double2 sg = zero;
        if (q < n) {
          const double2 bpq = A[p * N2 + q];
          const double bm2 = norm2(bpq);
          if (bm2 > 0.0) {
            const double x = A[q * N2 + q].x - A[p * N2 + p].x;
            const double ib = rsqrt(bm2);
            const double y2 = 4.0 * bm2;
            const double w = fabs(x) + sqrt(fma(x, x, y2));
            const double z = rsqrt(fma(w, w, y2));
            c = w * z;
            const double s = (x >= 0.0 ? 2.0 : -2.0) * (bm2 * ib) * z;  // sign(x) y z
            sg = make_double2(s * (bpq.x * ib), s * (bpq.y * ib));
          }
        }
        prm[2 * lane] = make_double2(c, 0.0);
        prm[2 * lane + 1] = sg;
      }
      wave_sync();
      const bool last = round == N2 - 2;
#pragma unroll
      for (int k = 0; k < L::TPL; ++k) {
        const int code = task[k];
        if (code < 0) continue;
        const bool is_v = code >= (1 << 16);
        const int i = (code >> 8) & 0xff, j = code & 0xff;
        const uint2 d = L::kTable ? ent[round * L::NT + lane + 64 * k] : task_entries<NP>(lane + 64 * k, round);
        const double cj = prm[2 * j].x;
        const double2 sj = prm[2 * j + 1];
        const double ci = is_v ? 1.0 : prm[2 * i].x;
        const double2 si = is_v ? zero : prm[2 * i + 1];
        // A holds its upper triangle only: an entry below the diagonal is the
        // conjugate of its transpose (flagged in its descriptor)
        double2 x00 = ld_entry(slice, d.x & 0xffff), x01 = ld_entry(slice, d.x >> 16);
        double2 x10 = ld_entry(slice, d.y & 0xffff), x11 = ld_entry(slice, d.y >> 16);
        rot_right(x00, x01, cj, sj);
        rot_right(x10, x11, cj, sj);
        rot_left(x00, x10, ci, si);
        rot_left(x01, x11, ci, si);
        const bool diag = !is_v && i == j;
        if (diag) {
          // a Hermitian 2x2 block: real diagonal; the plane's pair is annihilated exactly
          x00.y = 0.0;
          x11.y = 0.0;
          if (norm2(si) > 0.0) {
            x01 = zero;
            x10 = zero;
          } else {
            x10 = make_double2(x01.x, -x01.y);
          }
        }
        st_entry(slice, d.x & 0xffff, x00);
        st_entry(slice, d.x >> 16, x01);
        st_entry(slice, d.y & 0xffff, x10);
        st_entry(slice, d.y >> 16, x11);
        if (last && !is_v) {
          const double d = norm2(x00) + norm2(x11), o = norm2(x01) + norm2(x10);
          tot += diag ? d + o : 2.0 * (d + o);
          off += diag ? o : 2.0 * (d + o);
        }
      }
      wave_sync();
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    converged = off <= tol2 * tot;
    off = 0.0;
    tot = 0.0;
  }
  if (!converged && lane == 0) atomicOr(status, kStatusNoConv);
  // ascending order (ties by index), then each column's largest entry made real positive
  if (lane < n) {
    const double li = A[lane * N2 + lane].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * N2 + j].x;
      rank += (lj < li) || (lj == li && j < lane);
    }
    perm[rank] = lane;
  }
  wave_sync();
  if (lane < n) {
    const int src = perm[lane];
    eps[b * n + lane] = A[src * N2 + src].x;
    double best = -1.0;
    double2 bv = make_double2(1.0, 0.0);
    for (int r = 0; r < n; ++r) {
      const double2 v = V[r * N2 + src];
      const double m = norm2(v);
      if (m > best) {
        best = m;
        bv = v;
      }
    }
    const double mag = sqrt(best);
    fix[lane] = mag > 0.0 ? make_double2(bv.x / mag, -bv.y / mag) : make_double2(1.0, 0.0);
  }
  wave_sync();
  double2* out = reinterpret_cast<double2*>(Vout) + b * n * n;
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    const double2 v = V[r * N2 + perm[c]], f = fix[c];
    out[e] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
  }
}

// The solve for orders with one task per lane (n <= 12): A and V in position
// order, so every round loads and stores at the same per-lane offsets with
// no per-round descriptors (about a fifth fewer instructions per round).
// Larger orders keep the per-round descriptor tables: holding all of a
// lane's tasks in registers across the round would cost their occupancy.
template <int NP>
__device__ __forceinline__ void jacobi_small_body_pos(const double* __restrict__ H, int n, double* __restrict__ eps,
                                                  double* __restrict__ Vout, uint32_t* status, double tol2, int64_t b,
                                                  double2* slice, int lane) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2, TPL = L::TPL;
  double2* A = slice;
  double2* V = A + L::a_elems;
  double2* prm = V + L::a_elems;
  double2* fix = prm + L::prm_elems;
  int* perm = reinterpret_cast<int*>(fix + L::fix_elems);
  const double2* h = reinterpret_cast<const double2*>(H) + b * n * n;
  const double2 zero = make_double2(0.0, 0.0);

  // this lane's tasks: block (i, j) of A (i <= j) or of V, i.e. rows
  // {i, N2-1-i} x columns {j, N2-1-j} in position order (V: rows are the
  // basis, paired the same way), with the four entries' load offsets and the
  // offsets they are stored to (their positions in the next round)
  int task[TPL];
  uint2 ldo[TPL], sto[TPL];
#pragma unroll
  for (int k = 0; k < TPL; ++k) {
    const int t = lane + 64 * k;
    int code = -1;
    uint32_t l[4] = {0, 0, 0, 0}, w[4] = {0, 0, 0, 0};
    if (t < L::NT) {
      bool is_v;
      int i, j;
      decode_task<NP>(t, is_v, i, j);
      code = (is_v ? 1 << 16 : 0) | (i << 8) | j;
      const int rr[2] = {i, N2 - 1 - i}, cc[2] = {j, N2 - 1 - j};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = rr[e >> 1], c = cc[e & 1];
        l[e] = entry_offset<NP>(is_v, r, c);
        w[e] = entry_offset<NP>(is_v, is_v ? r : next_pos(r, N2), next_pos(c, N2));
      }
    }
    task[k] = code;
    ldo[k] = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
    sto[k] = make_uint2(w[0] | w[1] << 16, w[2] | w[3] << 16);
  }

  double off = 0.0, tot = 0.0;
  for (int e = lane; e < N2 * N2; e += 64) {
    const int r = e / N2, c = e % N2;
    const double2 v = (r < n && c < n) ? h[r * n + c] : zero;
    A[e] = v;
    V[e] = (r == c && r < n) ? make_double2(1.0, 0.0) : zero;
    const double m = norm2(v);
    tot += m;
    off += r != c ? m : 0.0;
  }
  off = wave_sum(off);
  tot = wave_sum(tot);
  wave_sync();
  bool converged = n <= 1 || off <= tol2 * tot;
  off = 0.0;
  tot = 0.0;
  const int max_sweeps = sweep_limit(status);
  for (int sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
#pragma unroll 1
    for (int round = 0; round < N2 - 1; ++round) {
      if (lane < NP) {
        // pair `lane`: positions p = lane, q = N2-1-lane (a zero padding
        // row and column give b = 0, the identity)
        const int p = lane, q = N2 - 1 - lane;
        double c = 1.0;
        double2 sg = zero;
        const double2 bpq = A[p * N2 + q];
        const double bm2 = norm2(bpq);
        if (bm2 > 0.0) {
          const double x = A[q * N2 + q].x - A[p * N2 + p].x;
          const double ib = rsqrt(bm2);
          const double y2 = 4.0 * bm2;
          const double w = fabs(x) + sqrt(fma(x, x, y2));
          const double z = rsqrt(fma(w, w, y2));
          c = w * z;
          const double s = (x >= 0.0 ? 2.0 : -2.0) * (bm2 * ib) * z;  // sign(x) y z
          sg = make_double2(s * (bpq.x * ib), s * (bpq.y * ib));
        }
        prm[2 * lane] = make_double2(c, 0.0);
        prm[2 * lane + 1] = sg;
      }
      wave_sync();
      const bool last = round == N2 - 2;
      // every entry is read before any is written (the stores go to the
      // moved positions, which other tasks read in this round)
      double2 x[TPL][4];
#pragma unroll
      for (int k = 0; k < TPL; ++k) {
        if (task[k] < 0) continue;
        x[k][0] = ld_entry(slice, ldo[k].x & 0xffff);
        x[k][1] = ld_entry(slice, ldo[k].x >> 16);
        x[k][2] = ld_entry(slice, ldo[k].y & 0xffff);
        x[k][3] = ld_entry(slice, ldo[k].y >> 16);
      }
#pragma unroll
      for (int k = 0; k < TPL; ++k) {
        const int code = task[k];
        if (code < 0) continue;
        const bool is_v = code >= (1 << 16);
        const int i = (code >> 8) & 0xff, j = code & 0xff;
        const double cj = prm[2 * j].x;
        const double2 sj = prm[2 * j + 1];
        const double ci = is_v ? 1.0 : prm[2 * i].x;
        const double2 si = is_v ? zero : prm[2 * i + 1];
        double2 x00 = x[k][0], x01 = x[k][1], x10 = x[k][2], x11 = x[k][3];
        rot_right(x00, x01, cj, sj);
        rot_right(x10, x11, cj, sj);
        rot_left(x00, x10, ci, si);
        rot_left(x01, x11, ci, si);
        const bool diag = !is_v && i == j;
        if (diag) {
          // a Hermitian 2x2 block: real diagonal; the plane's pair is annihilated exactly
          x00.y = 0.0;
          x11.y = 0.0;
          if (norm2(si) > 0.0) {
            x01 = zero;
            x10 = zero;
          } else {
            x10 = make_double2(x01.x, -x01.y);
          }
        }
        st_entry(slice, sto[k].x & 0xffff, x00);
        st_entry(slice, sto[k].x >> 16, x01);
        st_entry(slice, sto[k].y & 0xffff, x10);
        st_entry(slice, sto[k].y >> 16, x11);
        if (last && !is_v) {
          const double d = norm2(x00) + norm2(x11), o = norm2(x01) + norm2(x10);
          tot += diag ? d + o : 2.0 * (d + o);
          off += diag ? o : 2.0 * (d + o);
        }
      }
      wave_sync();
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    converged = off <= tol2 * tot;
    off = 0.0;
    tot = 0.0;
  }
  if (!converged && lane == 0) atomicOr(status, kStatusNoConv);
  // ascending order (ties by index), then each column's largest entry made real positive
  if (lane < n) {
    const double li = A[lane * N2 + lane].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = A[j * N2 + j].x;
      rank += (lj < li) || (lj == li && j < lane);
    }
    perm[rank] = lane;
  }
  wave_sync();
  if (lane < n) {
    const int src = perm[lane];
    eps[b * n + lane] = A[src * N2 + src].x;
    double best = -1.0;
    double2 bv = make_double2(1.0, 0.0);
    for (int r = 0; r < n; ++r) {
      const double2 v = V[r * N2 + src];
      const double m = norm2(v);
      if (m > best) {
        best = m;
        bv = v;
      }
    }
    const double mag = sqrt(best);
    fix[lane] = mag > 0.0 ? make_double2(bv.x / mag, -bv.y / mag) : make_double2(1.0, 0.0);
  }
  wave_sync();
  double2* out = reinterpret_cast<double2*>(Vout) + b * n * n;
  for (int e = lane; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    const double2 v = V[r * N2 + perm[c]], f = fix[c];
    out[e] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
  }
}

// blockDim.x / 64 matrices per workgroup, one wavefront each: a CU's
// workgroup slots would otherwise cap it at one single-wave solve per slot
template <int NP>
__global__ void __launch_bounds__(64 * kSmallPerBlock)
    jacobi_small_kernel(const double* __restrict__ H, int64_t batch, int n, double* __restrict__ eps,
                        double* __restrict__ V, uint32_t* status, double tol2) {
  extern __shared__ double2 jlds[];
  using L = SmallLayout<NP>;
  const int wave = threadIdx.x >> 6, per = blockDim.x >> 6;
  uint2* ent = reinterpret_cast<uint2*>(jlds + per * L::slice_elems);
  int* pqt = reinterpret_cast<int*>(ent + (L::N2 - 1) * L::NT);
  if (L::kTable) {
    build_tables<NP>(ent, pqt);
    __syncthreads();
  }
  const int64_t m = (int64_t)blockIdx.x * per + wave;
  if (m >= batch) return;
  if constexpr (L::TPL == 1)
    jacobi_small_body_pos<NP>(H, n, eps, V, status, tol2, m, jlds + wave * L::slice_elems, threadIdx.x & 63);
  else
    jacobi_small_body<NP>(H, n, eps, V, status, tol2, m, jlds + wave * L::slice_elems, threadIdx.x & 63, ent, pqt);
}

// NP covers the largest order among the jobs; smaller orders run padded
template <int NP>
__global__ void __launch_bounds__(64 * kSmallPerBlock)
    jacobi_grouped_kernel(const EighJob* __restrict__ jobs, int njobs, int64_t total, uint32_t* status) {
  extern __shared__ double2 jlds[];
  using L = SmallLayout<NP>;
  const int wave = threadIdx.x >> 6, per = blockDim.x >> 6;
  uint2* ent = reinterpret_cast<uint2*>(jlds + per * L::slice_elems);
  int* pqt = reinterpret_cast<int*>(ent + (L::N2 - 1) * L::NT);
  if (L::kTable) {
    build_tables<NP>(ent, pqt);
    __syncthreads();
  }
  const int64_t m = (int64_t)blockIdx.x * per + wave;
  if (m >= total) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_base <= m) lo = mid; else hi = mid - 1;
  }
  const EighJob& j = jobs[lo];
  if constexpr (L::TPL == 1)
    jacobi_small_body_pos<NP>(j.H, j.n, j.eps, j.V, status, kOffTol2, m - j.block_base,
                              jlds + wave * L::slice_elems, threadIdx.x & 63);
  else
    jacobi_small_body<NP>(j.H, j.n, j.eps, j.V, status, kOffTol2, m - j.block_base, jlds + wave * L::slice_elems,
                          threadIdx.x & 63, ent, pqt);
}

using SmallKernel = void (*)(const double*, int64_t, int, double*, double*, uint32_t*, double);
using GroupedKernel = void (*)(const EighJob*, int, int64_t, uint32_t*);

template <int... NPs>
struct SmallTable {
  static SmallKernel small(int np) {
    SmallKernel k = nullptr;
    ((np == NPs ? (k = jacobi_small_kernel<NPs>, 0) : 0), ...);
    return k;
  }
  static GroupedKernel grouped(int np) {
    GroupedKernel k = nullptr;
    ((np == NPs ? (k = jacobi_grouped_kernel<NPs>, 0) : 0), ...);
    return k;
  }
  // solves per workgroup: up to kSmallPerBlock within the 64 KB of dynamic LDS
  static int per_block(int np) {
    size_t v = 0, t = 0;
    ((np == NPs ? (v = SmallLayout<NPs>::slice_elems * 16, t = SmallLayout<NPs>::table_elems * 16, 0) : 0), ...);
    const size_t fit = v ? (65536 - t) / v : 1;
    return (int)(fit < (size_t)kSmallPerBlock ? (fit ? fit : 1) : kSmallPerBlock);
  }
  static size_t bytes(int np) {
    size_t v = 0, t = 0;
    ((np == NPs ? (v = SmallLayout<NPs>::slice_elems * 16, t = SmallLayout<NPs>::table_elems * 16, 0) : 0), ...);
    return v * per_block(np) + t;
  }
};
using Small = SmallTable<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16>;

// one workgroup of 16 waves per large matrix: the rounds stream A and V
// through the caches (640 KB each at n = 200), so the more loads in flight
// the better; the rotation parameters stay in LDS
constexpr int kLargeThreads = 1024;

__global__ void __launch_bounds__(kLargeThreads)
    jacobi_large_kernel(const double* __restrict__ H, int n, double* __restrict__ eps,
                        double* __restrict__ V, double* __restrict__ work, uint32_t* status) {
  __shared__ double rc[128], rs[128], rer[128], rei[128], phr[256], phi[256], red[kLargeThreads / 64];
  __shared__ int rp[128], rq[128], perm[256];
  const int64_t b = blockIdx.x;
  const int64_t nn = (int64_t)n * n;
  double* Ar = work + 4 * nn * blockIdx.x;
  double* Ai = Ar + nn;
  double* Vr = Ai + nn;
  double* Vi = Vr + nn;
  const double* h = H + 2 * b * nn;
  for (int64_t e = threadIdx.x; e < nn; e += kLargeThreads) {
    Ar[e] = h[2 * e];
    Ai[e] = h[2 * e + 1];
  }
  __syncthreads();
  const bool ok = jacobi_core<kLargeThreads>(Ar, Ai, Vr, Vi, n, rc, rs, rer, rei, rp, rq, red, sweep_limit(status));
  if (!ok && threadIdx.x == 0) atomicOr(status, kStatusNoConv);
  jacobi_finish<kLargeThreads>(Ar, Vr, Vi, n, perm, phr, phi, eps + b * n, V + 2 * b * nn);
}

constexpr int64_t kLargeChunk = 1024;  // matrices per large-n launch (bounds the workspace)

}  // namespace

int64_t jacobi_work_doubles(int n, int64_t batch) {
  if (n <= kSmallN) return 0;
  const int64_t chunk = batch < kLargeChunk ? batch : kLargeChunk;
  return 4 * (int64_t)n * n * chunk;
}

ephw_status jacobi_eigh_grouped(const EighJob* d_jobs, int njobs, int64_t total, int max_n, uint32_t* status,
                                hipStream_t s) {
  if (njobs <= 0 || total <= 0) return EPHW_OK;
  if (max_n < 1 || max_n > kSmallN) {
    set_error("jacobi_eigh_grouped: matrix orders must be in [1, 32]");
    return EPHW_EUNSUPPORTED;
  }
  const int np = (max_n + 1) / 2, per = Small::per_block(np);
  const int64_t grid = (total + per - 1) / per;
  if (grid > 0x7fffffff) {
    set_error("jacobi_eigh_grouped: too many matrices for one launch");
    return EPHW_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(Small::grouped(np), dim3((unsigned)grid), dim3(64 * per), Small::bytes(np), s, d_jobs, njobs,
                     total, status);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status jacobi_eigh(const double* H, int64_t batch, int n, double* eps, double* V, double* work,
                        uint32_t* status, hipStream_t s, double off_tol2) {
  if (batch <= 0) return EPHW_OK;
  if (!(off_tol2 > 0.0) || off_tol2 < kOffTol2) off_tol2 = kOffTol2;
  if ((reinterpret_cast<uintptr_t>(H) | reinterpret_cast<uintptr_t>(V)) & 15) {
    set_error("jacobi_eigh: matrices and eigenvectors must be 16-byte aligned complex128 arrays");
    return EPHW_EINVAL;
  }
  if (n < 1 || n > 256) {
    set_error("jacobi_eigh: matrix order must be in [1, 256]");
    return EPHW_EUNSUPPORTED;
  }
  if (n <= kSmallN) {
    const int np = (n + 1) / 2, per = Small::per_block(np);
    const int64_t max_per_launch = (int64_t)0x7fffffff * per;
    for (int64_t b0 = 0; b0 < batch; b0 += max_per_launch) {
      const int64_t nb = (batch - b0) < max_per_launch ? (batch - b0) : max_per_launch;
      const int64_t grid = (nb + per - 1) / per;
      hipLaunchKernelGGL(Small::small(np), dim3((unsigned)grid), dim3(64 * per), Small::bytes(np), s,
                         H + 2 * b0 * n * n, nb, n, eps + b0 * n, V + 2 * b0 * n * n, status, off_tol2);
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
    hipLaunchKernelGGL(jacobi_large_kernel, dim3((unsigned)nb), dim3(kLargeThreads), 0, s,
                       H + 2 * b0 * (int64_t)n * n, n, eps + b0 * n, V + 2 * b0 * (int64_t)n * n,
                       work, status);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

}  // namespace ephw
