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
// Small matrices (n <= 32) live in LDS sized to the order (4 KB per solve at
// n = 11) so that a CU holds as many solves as its registers allow; each lane
// owns one 2x2 block of the round (below), a wavefront runs one solve, or
// several up to n = 12.  Large matrices (n > 32) live in a global workspace,
// one 1024-thread workgroup per matrix (the rotation parameters stay in LDS).
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
// Small solves (n <= 32): a 64-lane wavefront per matrix (several matrices
// up to n = 12, below), A and V in LDS as
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
//   c = w z, s = sign(x) y z, sigma = s b/|b| = sign(x) 2 z b,
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
  // A and V: the full squares, or, where the solve keeps per-lane offsets
  // (one task per lane), task-major: entry e of task t's block at e RS + t,
  // the regions RS apart (an odd stride above 32 tasks, which spreads the
  // scattered stores to the moved positions over more LDS banks)
  static constexpr bool kTaskMajor = TPL == 1;
  static constexpr int RS = NT > 32 ? 63 : NT;
  static constexpr size_t data_elems = kTaskMajor ? 3 * (size_t)RS + NT : 2 * a_elems;
  static constexpr size_t prm_elems = 2 * (size_t)NP;            // per pair (c, 0), sigma; task-major: sigma[NP], c[NP]
  static constexpr size_t fix_elems = (size_t)N2;                // phase fix per column
  static constexpr size_t bytes = (data_elems + prm_elems + fix_elems) * 16 + (size_t)N2 * 4;
  static constexpr size_t slice_elems = (bytes + 15) / 16;       // one wavefront's share, 16-byte units
  // per-round task descriptors and plane pairs, shared by the workgroup's
  // solves (which all have this padded order), when they fit
  static constexpr size_t table_bytes = (size_t)(N2 - 1) * NT * 8 + (size_t)(N2 - 1) * NP * 4;
  static constexpr bool kTable = TPL > 1 && table_bytes <= 32768;
  static constexpr size_t table_elems = kTable ? (table_bytes + 15) / 16 : 0;
};

template <int NP>
__host__ __device__ __forceinline__ void decode_task(int t, bool& is_v, int& i, int& j) {
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
__host__ __device__ __forceinline__ int next_pos(int pos, int n2) {
  return pos == 0 ? 0 : (pos == 1 ? n2 - 1 : pos - 1);
}

// Where entries live in the one-task-per-lane solves: entry e (0..3, row
// bit then column bit) of task t's block at e RS + t, so that each of a
// round's four loads reads consecutive lanes' entries from consecutive
// addresses (no LDS bank conflicts).  In position order the entry (r, c)
// belongs to the planes pr(r), pr(c) of its row and column (pr(x) = x below
// NP, else N2 - 1 - x), at row bit r >= NP and column bit c >= NP.  A keeps
// one slot per entry of its upper triangle: an entry below the diagonal is
// read and written as the conjugate of its transpose (bit 15 of the offset).
// V: task NA + pr(r) NP + pr(c).  A, (r, c) with r <= c, a = pr(r), b = pr(c):
// a < b: block (a, b); a > b: block (b, a), whose entry (c, r) lies below
// the diagonal and so holds this one; a = b: the diagonal block (a, a), whose
// entries (a, N2-1-a) and (N2-1-a, a) share slot 1.
template <int NP>
__host__ __device__ __forceinline__ uint32_t entry_offset(bool is_v, int r, int c) {
  using L = SmallLayout<NP>;
  constexpr int N2 = L::N2, RS = L::RS, NA = L::NA;
  const auto pr = [](int x) { return x < NP ? x : N2 - 1 - x; };
  const auto hi = [](int x) { return x >= NP ? 1 : 0; };
  // task of A block (a, b), a <= b: the blocks are numbered row by row
  const auto task_a = [](int a, int b) { return a * NP - a * (a - 1) / 2 + (b - a); };
  if (is_v) return (uint32_t)((2 * hi(r) + hi(c)) * RS + NA + pr(r) * NP + pr(c));
  uint32_t flag = 0;
  if (r > c) {
    const int t = r;
    r = c;
    c = t;
    flag = 0x8000u;
  }
  const int a = pr(r), b = pr(c);
  int e, t;
  if (a < b) {
    e = 2 * hi(r) + hi(c);
    t = task_a(a, b);
  } else if (a > b) {
    e = 2 * hi(c) + hi(r);
    t = task_a(b, a);
  } else {
    e = r == c ? 3 * hi(r) : 1;
    t = task_a(a, a);
  }
  return (uint32_t)(e * RS + t) | flag;
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
    double2 v = (r < n && c < n) ? h[r * n + c] : zero;
    if (r == c) v.y = 0.0;  // Hermitian: a real diagonal
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
            const double y2 = 4.0 * bm2;
            const double w = fabs(x) + sqrt(fma(x, x, y2));
            const double z = rsqrt(fma(w, w, y2));
            c = w * z;
            const double f = (x >= 0.0 ? 2.0 : -2.0) * z;  // sigma = sign(x) y z b/|b| = sign(x) 2 z b
            sg = make_double2(f * bpq.x, f * bpq.y);
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
          // a rotated Hermitian 2x2 block: real diagonal, the plane's pair
          // annihilated exactly (an unrotated one keeps its entries bit for bit)
          if (norm2(si) > 0.0) {
            x00.y = 0.0;
            x11.y = 0.0;
            x01 = zero;
            x10 = zero;
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
//
// A wavefront runs several such solves: G lane groups of LPM lanes (the
// tasks of one solve, rounded up to a power of two) and S solves per group,
// whose blocks a lane updates one after the other with the same offsets.
// The plane parameters of the group's S solves come from S NP lanes at once,
// so the instructions of that step (about a third of a round's with one solve
// per wavefront) serve S solves.  The wavefront sweeps until all its solves have
// converged; a converged solve takes identity rotations (c = 1, sigma = 0,
// which leave every entry unchanged) and only moves its entries through the
// positions, so its results do not depend on the solves beside it.
template <int NP>
struct PosShape {
  static constexpr int NT = SmallLayout<NP>::NT;
  static constexpr int LPM = NT <= 2 ? 2 : NT <= 4 ? 4 : NT <= 8 ? 8 : NT <= 16 ? 16 : NT <= 32 ? 32 : 64;
  static constexpr int G = 64 / LPM;
  static constexpr int S = 2;
  static constexpr int M = G * S;  // solves per wavefront
  static_assert(S * NP <= LPM && 2 * NP <= LPM, "a group's lanes must cover its plane parameters and its order");
};

template <int NP>
constexpr int solves_per_wave() {
  if constexpr (SmallLayout<NP>::TPL == 1) return PosShape<NP>::M;
  else return 1;
}

// one solve of a wavefront: matrix b of H (n x n), its outputs; n = 0: none
struct PosJob {
  const double* H;
  double* eps;
  double* V;
  int64_t b;
  int n;
};

template <int LPM>
__device__ __forceinline__ double group_sum(double v) {
  for (int m = LPM / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// job_at(s): the group's solve s (called before the sweeps and again for the
// outputs, so that no job is held in registers across them); slices: the
// group's S solve slices, one after the other; lg: lane in group
template <int NP, class JobAt>
__device__ __forceinline__ void jacobi_small_body_pos(JobAt job_at, uint32_t* status, double tol2, double2* slices,
                                                      int lg) {
  using L = SmallLayout<NP>;
  using P = PosShape<NP>;
  constexpr int N2 = L::N2, S = P::S, LPM = P::LPM;
  constexpr size_t SL = L::slice_elems, PO = L::data_elems;
  static_assert(L::kTaskMajor, "the one-task-per-lane solve keeps A and V task-major");
  // entry (r, c) of A (r <= c, no conjugate flag) or of V
  const auto at_a = [](int r, int c) { return entry_offset<NP>(false, r, c); };
  const auto at_v = [](int r, int c) { return entry_offset<NP>(true, r, c); };
  const double2 zero = make_double2(0.0, 0.0);

  // this lane's task: block (i, j) of A (i <= j) or of V, i.e. rows
  // {i, N2-1-i} x columns {j, N2-1-j} in position order (V: rows are the
  // basis, paired the same way), with the four entries' load offsets and the
  // offsets they are stored to (their positions in the next round); the
  // same in each of the group's solves
  int code = -1;
  uint2 ldo = make_uint2(0, 0), sto = make_uint2(0, 0);
  if (lg < L::NT) {
    bool is_v;
    int i, j;
    decode_task<NP>(lg, is_v, i, j);
    code = (is_v ? 1 << 16 : 0) | (i << 8) | j;
    const int rr[2] = {i, N2 - 1 - i}, cc[2] = {j, N2 - 1 - j};
    uint32_t l[4], w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rr[e >> 1], c = cc[e & 1];
      l[e] = entry_offset<NP>(is_v, r, c);
      w[e] = entry_offset<NP>(is_v, is_v ? r : next_pos(r, N2), next_pos(c, N2));
    }
    ldo = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
    sto = make_uint2(w[0] | w[1] << 16, w[2] | w[3] << 16);
  }
  const bool is_v = code >= (1 << 16);
  const int ti = (code >> 8) & 0xff, tj = code & 0xff;
  const bool diag = code >= 0 && !is_v && ti == tj;

  bool conv[S];
  double off[S], tot[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double2* X = slices + s * SL;
    const PosJob job = job_at(s);
    const int n = job.n;
    const double2* h = reinterpret_cast<const double2*>(job.H) + job.b * n * n;
    double o = 0.0, t = 0.0;
    for (int e = lg; e < N2 * N2; e += LPM) {
      const int r = e / N2, c = e % N2;
      double2 v = (r < n && c < n) ? h[r * n + c] : zero;
      if (r == c) v.y = 0.0;  // Hermitian: a real diagonal
      if (r <= c) X[at_a(r, c)] = v;
      X[at_v(r, c)] = (r == c && r < n) ? make_double2(1.0, 0.0) : zero;
      const double m = norm2(v);
      t += m;
      o += r != c ? m : 0.0;
    }
    o = group_sum<LPM>(o);
    t = group_sum<LPM>(t);
    conv[s] = n <= 1 || o <= tol2 * t;
    off[s] = 0.0;
    tot[s] = 0.0;
  }
  wave_sync();
  const int max_sweeps = sweep_limit(status);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    bool all = true;
#pragma unroll
    for (int s = 0; s < S; ++s) all = all && conv[s];
    if (__all(all)) break;
#pragma unroll 1
    for (int round = 0; round < N2 - 1; ++round) {
      if (lg < S * NP) {
        // pair k of solve s: positions p = k, q = N2-1-k (a zero padding row
        // and column give b = 0, the identity)
        const int s = lg / NP, k = lg - s * NP;
        double2* A = slices + s * SL;
        double2* prm = A + PO;
        bool done = conv[0];
#pragma unroll
        for (int u = 1; u < S; ++u) done = s == u ? conv[u] : done;
        const int p = k, q = N2 - 1 - k;
        double c = 1.0;
        double2 sg = zero;
        const double2 bpq = A[at_a(p, q)];
        const double bm2 = norm2(bpq);
        if (!done && bm2 > 0.0) {
          const double x = A[at_a(q, q)].x - A[at_a(p, p)].x;
          const double y2 = 4.0 * bm2;
          const double w = fabs(x) + sqrt(fma(x, x, y2));
          const double z = rsqrt(fma(w, w, y2));
          c = w * z;
          const double f = (x >= 0.0 ? 2.0 : -2.0) * z;  // sigma = sign(x) y z b/|b| = sign(x) 2 z b
          sg = make_double2(f * bpq.x, f * bpq.y);
        }
        prm[k] = sg;
        reinterpret_cast<double*>(prm + NP)[k] = c;
      }
      wave_sync();
      const bool last = round == N2 - 2;
      // every entry is read before any is written (the stores go to the
      // moved positions, which other tasks read in this round)
      double2 x[S][4];
      if (code >= 0) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const double2* X = slices + s * SL;
          x[s][0] = ld_entry(X, ldo.x & 0xffff);
          x[s][1] = ld_entry(X, ldo.x >> 16);
          x[s][2] = ld_entry(X, ldo.y & 0xffff);
          x[s][3] = ld_entry(X, ldo.y >> 16);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
          double2* X = slices + s * SL;
          // sigma of the NP planes, then their c: consecutive planes' parameters
          // in consecutive LDS banks
          const double2* prm = X + PO;
          const double* pc = reinterpret_cast<const double*>(prm + NP);
          const double cj = pc[tj];
          const double2 sj = prm[tj];
          const double ci = is_v ? 1.0 : pc[ti];
          const double2 si = is_v ? zero : prm[ti];
          double2 x00 = x[s][0], x01 = x[s][1], x10 = x[s][2], x11 = x[s][3];
          rot_right(x00, x01, cj, sj);
          rot_right(x10, x11, cj, sj);
          rot_left(x00, x10, ci, si);
          rot_left(x01, x11, ci, si);
          if (diag) {
            // a rotated Hermitian 2x2 block: real diagonal, the plane's pair
            // annihilated exactly (an unrotated one keeps its entries bit for bit)
            if (norm2(si) > 0.0) {
              x00.y = 0.0;
              x11.y = 0.0;
              x01 = zero;
              x10 = zero;
            }
          }
          st_entry(X, sto.x & 0xffff, x00);
          st_entry(X, sto.x >> 16, x01);
          st_entry(X, sto.y & 0xffff, x10);
          st_entry(X, sto.y >> 16, x11);
          if (last && !is_v) {
            const double d = norm2(x00) + norm2(x11), o = norm2(x01) + norm2(x10);
            tot[s] += diag ? d + o : 2.0 * (d + o);
            off[s] += diag ? o : 2.0 * (d + o);
          }
        }
      }
      wave_sync();
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const double o = group_sum<LPM>(off[s]), t = group_sum<LPM>(tot[s]);
      conv[s] = conv[s] || o <= tol2 * t;
      off[s] = 0.0;
      tot[s] = 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (!conv[s] && lg == 0) atomicOr(status, kStatusNoConv);
  // ascending order (ties by index), then each column's largest entry made real positive
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double2* A = slices + s * SL;
    int* perm = reinterpret_cast<int*>(A + PO + L::prm_elems + L::fix_elems);
    const int n = job_at(s).n;
    if (lg < n) {
      const double li = A[at_a(lg, lg)].x;
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const double lj = A[at_a(j, j)].x;
        rank += (lj < li) || (lj == li && j < lg);
      }
      perm[rank] = lg;
    }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    double2* A = slices + s * SL;
    double2* fix = A + PO + L::prm_elems;
    const int* perm = reinterpret_cast<const int*>(fix + L::fix_elems);
    const PosJob job = job_at(s);
    const int n = job.n;
    if (lg < n) {
      const int src = perm[lg];
      job.eps[job.b * n + lg] = A[at_a(src, src)].x;
      double best = -1.0;
      double2 bv = make_double2(1.0, 0.0);
      for (int r = 0; r < n; ++r) {
        const double2 v = A[at_v(r, src)];
        const double m = norm2(v);
        if (m > best) {
          best = m;
          bv = v;
        }
      }
      const double mag = sqrt(best);
      fix[lg] = mag > 0.0 ? make_double2(bv.x / mag, -bv.y / mag) : make_double2(1.0, 0.0);
    }
  }
  wave_sync();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double2* A = slices + s * SL;
    const double2* fix = A + PO + L::prm_elems;
    const int* perm = reinterpret_cast<const int*>(fix + L::fix_elems);
    const PosJob job = job_at(s);
    const int n = job.n;
    double2* out = reinterpret_cast<double2*>(job.V) + job.b * n * n;
    for (int e = lg; e < n * n; e += LPM) {
      const int r = e / n, c = e % n;
      const double2 v = A[at_v(r, perm[c])], f = fix[c];
      out[e] = make_double2(v.x * f.x - v.y * f.y, v.x * f.y + v.y * f.x);
    }
  }
}

// blockDim.x / 64 wavefronts per workgroup, each with solves_per_wave<NP>()
// solves: a CU's workgroup slots would otherwise cap it at one single-wave
// solve per slot
template <int NP>
__global__ void __launch_bounds__(64 * kSmallPerBlock)
    jacobi_small_kernel(const double* __restrict__ H, int64_t batch, int n, double* __restrict__ eps,
                        double* __restrict__ V, uint32_t* status, double tol2) {
  extern __shared__ double2 jlds[];
  using L = SmallLayout<NP>;
  constexpr int M = solves_per_wave<NP>();
  const int wave = threadIdx.x >> 6, per = blockDim.x >> 6;
  uint2* ent = reinterpret_cast<uint2*>(jlds + per * M * L::slice_elems);
  int* pqt = reinterpret_cast<int*>(ent + (L::N2 - 1) * L::NT);
  if (L::kTable) {
    build_tables<NP>(ent, pqt);
    __syncthreads();
  }
  const int64_t m0 = ((int64_t)blockIdx.x * per + wave) * M;
  if (m0 >= batch) return;
  const int lane = threadIdx.x & 63;
  if constexpr (L::TPL == 1) {
    using P = PosShape<NP>;
    const int g = lane / P::LPM;
    const int64_t mg = m0 + g * P::S;
    auto job_at = [=](int s) {
      const int64_t m = mg + s;
      return PosJob{H, eps, V, m < batch ? m : 0, m < batch ? n : 0};
    };
    jacobi_small_body_pos<NP>(job_at, status, tol2, jlds + (wave * M + g * P::S) * L::slice_elems, lane % P::LPM);
  } else {
    jacobi_small_body<NP>(H, n, eps, V, status, tol2, m0, jlds + wave * L::slice_elems, lane, ent, pqt);
  }
}

__device__ __forceinline__ int find_job(const EighJob* __restrict__ jobs, int njobs, int64_t m) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_base <= m) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// NP covers the largest order among the jobs; smaller orders run padded
template <int NP>
__global__ void __launch_bounds__(64 * kSmallPerBlock)
    jacobi_grouped_kernel(const EighJob* __restrict__ jobs, int njobs, int64_t total, uint32_t* status) {
  extern __shared__ double2 jlds[];
  using L = SmallLayout<NP>;
  constexpr int M = solves_per_wave<NP>();
  const int wave = threadIdx.x >> 6, per = blockDim.x >> 6;
  uint2* ent = reinterpret_cast<uint2*>(jlds + per * M * L::slice_elems);
  int* pqt = reinterpret_cast<int*>(ent + (L::N2 - 1) * L::NT);
  if (L::kTable) {
    build_tables<NP>(ent, pqt);
    __syncthreads();
  }
  const int64_t m0 = ((int64_t)blockIdx.x * per + wave) * M;
  if (m0 >= total) return;
  const int lane = threadIdx.x & 63;
  if constexpr (L::TPL == 1) {
    using P = PosShape<NP>;
    const int g = lane / P::LPM;
    const int64_t mg = m0 + g * P::S;
    auto job_at = [=](int s) {
      const int64_t m = mg + s;
      if (m >= total) return PosJob{nullptr, nullptr, nullptr, 0, 0};
      const EighJob& j = jobs[find_job(jobs, njobs, m)];
      return PosJob{j.H, j.eps, j.V, m - j.block_base, j.n};
    };
    jacobi_small_body_pos<NP>(job_at, status, kOffTol2, jlds + (wave * M + g * P::S) * L::slice_elems,
                              lane % P::LPM);
  } else {
    const EighJob& j = jobs[find_job(jobs, njobs, m0)];
    jacobi_small_body<NP>(j.H, j.n, j.eps, j.V, status, kOffTol2, m0 - j.block_base, jlds + wave * L::slice_elems,
                          lane, ent, pqt);
  }
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
  static int per_wave(int np) {
    int m = 1;
    ((np == NPs ? (m = solves_per_wave<NPs>(), 0) : 0), ...);
    return m;
  }
  // wavefronts per workgroup: up to kSmallPerBlock, their solves within the
  // 64 KB of dynamic LDS
  static int per_block(int np) {
    size_t v = 0, t = 0;
    ((np == NPs ? (v = SmallLayout<NPs>::slice_elems * 16 * solves_per_wave<NPs>(),
                   t = SmallLayout<NPs>::table_elems * 16, 0)
                : 0),
     ...);
    const size_t fit = v ? (65536 - t) / v : 1;
    return (int)(fit < (size_t)kSmallPerBlock ? (fit ? fit : 1) : kSmallPerBlock);
  }
  static size_t bytes(int np) {
    size_t v = 0, t = 0;
    ((np == NPs ? (v = SmallLayout<NPs>::slice_elems * 16 * solves_per_wave<NPs>(),
                   t = SmallLayout<NPs>::table_elems * 16, 0)
                : 0),
     ...);
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
  const int np = (max_n + 1) / 2, waves = Small::per_block(np), per = waves * Small::per_wave(np);
  const int64_t grid = (total + per - 1) / per;
  if (grid > 0x7fffffff) {
    set_error("jacobi_eigh_grouped: too many matrices for one launch");
    return EPHW_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(Small::grouped(np), dim3((unsigned)grid), dim3(64 * waves), Small::bytes(np), s, d_jobs, njobs,
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
    const int np = (n + 1) / 2, waves = Small::per_block(np), per = waves * Small::per_wave(np);
    const int64_t max_per_launch = (int64_t)0x7fffffff * per;
    for (int64_t b0 = 0; b0 < batch; b0 += max_per_launch) {
      const int64_t nb = (batch - b0) < max_per_launch ? (batch - b0) : max_per_launch;
      const int64_t grid = (nb + per - 1) / per;
      hipLaunchKernelGGL(Small::small(np), dim3((unsigned)grid), dim3(64 * waves), Small::bytes(np), s,
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
