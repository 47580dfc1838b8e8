// Eq. (7) on an explicit list of (k, q) pairs: the pairs that survive the
// energy-window pre-screening the paper applies before interpolating.
//
// Eq. (7)'s double phase sum can be nested either way round.  Grouped by q
// (the paper's order, Eqs. (9)-(10)): per batch of q, the Rp sum of Eq. (9)
// over every Re as one GEMM and the mode vectors applied to g(Re,q); then,
// per q, the Re sum for that q's kept k only,
//   W_q[kept k][nu m' n'] = P_k[kept k][Re] G_nu(Re, q),
// with the P_k rows of the kept k gathered into a contiguous block.  Grouped
// by k: per chunk of k, the Re sum over every Rp first, as one GEMM batched
// over Rp,
//   G'(k, Rp)[ka m' n'] = sum_Re P_k[k][Re] g(Re, Rp),
// then, per k, the Rp sum for that k's kept q only,
//   W_k[kept q][ka m' n'] = P_q[kept q][Rp] G'(k, Rp),
// and the mode vectors u(q) per pair.  In both, the per-group sums are the
// problems of a grouped persistent GEMM (as many rows as the group has kept
// pairs), and the band rotations V(k+q)^dagger W V(k) and the epilogues run
// per pair in the band-rotation kernel's pair mode.  Outputs are indexed by
// pair, in the order of the list.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace ephw {
namespace {

// dst[i][:] = src[idx[i]][:] for complex rows of `width` values
template <typename T>
__global__ void gather_complex_rows_kernel(const T* __restrict__ src, int64_t nsrc, const int32_t* __restrict__ idx,
                                           int64_t width, T* __restrict__ dst, uint32_t* status) {
  const int64_t i = blockIdx.y;
  int64_t r = idx[i];
  if (r < 0 || r >= nsrc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, kStatusIndex);
    r = 0;
  }
  const T* s = src + 2 * r * width;
  T* d = dst + 2 * i * width;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < width; c += (int64_t)gridDim.x * blockDim.x) {
    d[2 * c] = s[2 * c];
    d[2 * c + 1] = s[2 * c + 1];
  }
}

template <typename T>
ephw_status gather_complex_rows(const void* src, int64_t nsrc, const int32_t* idx, int64_t cnt, int64_t width,
                                void* dst, uint32_t* status, hipStream_t st) {
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(width, 256), 64);
  for (int64_t c0 = 0; c0 < cnt; c0 += 65535) {
    const int64_t cn = std::min<int64_t>(65535, cnt - c0);
    hipLaunchKernelGGL(gather_complex_rows_kernel<T>, dim3(gx, (unsigned)cn), dim3(256), 0, st,
                       static_cast<const T*>(src), nsrc, idx + c0, width, static_cast<T*>(dst) + 2 * c0 * width,
                       status);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

// out[p] = val[i] for the pairs p of group i: [seg[i], seg[i+1])
__global__ void fill_segments_kernel(const int64_t* __restrict__ seg, const int32_t* __restrict__ val,
                                     int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x;
  const int32_t v = val[i];
  for (int64_t p = seg[i] + threadIdx.x; p < seg[i + 1]; p += blockDim.x) out[p] = v;
}

__global__ void gather_q_kernel(const double* __restrict__ q, const int32_t* __restrict__ qidx, int64_t n,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n) out[i] = q[3 * (int64_t)qidx[i / 3] + i % 3];
}

// Mode vectors per pair: out[p][nu][e] = sum_a W[p][a][e] u(q_p)[a][nu]
// (e over the Nw^2 band pairs), one thread per (pair, e).
template <typename T>
__global__ void pair_mode_rotate_kernel(const T* __restrict__ W, const T* __restrict__ u,
                                        const int32_t* __restrict__ pair_q, int64_t nq, int64_t npairs, int nm,
                                        int nw2, T* __restrict__ out, uint32_t* status) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npairs * nw2) return;
  const int64_t p = idx / nw2;
  const int e = (int)(idx % nw2);
  int64_t q = pair_q[p];
  if (q < 0 || q >= nq) {
    if (e == 0) atomicOr(status, kStatusIndex);
    q = 0;
  }
  const T* w = W + 2 * (p * nm * nw2 + e);
  const T* uq = u + 2 * q * nm * nm;
  T* o = out + 2 * (p * nm * nw2 + e);
  for (int v = 0; v < nm; ++v) {
    cplx<T> acc{0, 0};
    for (int a = 0; a < nm; ++a)
      cfma(acc, cplx<T>{w[2 * a * nw2], w[2 * a * nw2 + 1]}, cplx<T>{uq[2 * (a * nm + v)], uq[2 * (a * nm + v) + 1]});
    o[2 * v * nw2] = acc.re;
    o[2 * v * nw2 + 1] = acc.im;
  }
}

// pinned host staging of at least `bytes`, once the previous call's copy from it is done
ephw_status stage_reserve(ephw_system* s, size_t bytes) {
  if (s->staged) EPHW_HIP(hipEventSynchronize(s->staged));
  else EPHW_HIP(hipEventCreateWithFlags(&s->staged, hipEventDisableTiming));
  if (s->stage_bytes >= bytes && s->stage_host) return EPHW_OK;
  if (s->stage_host) EPHW_HIP(hipHostFree(s->stage_host));
  s->stage_host = nullptr;
  s->stage_bytes = 0;
  if (hipHostMalloc(&s->stage_host, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    s->stage_host = nullptr;
    set_error("pinned staging allocation of " + std::to_string(bytes) + " bytes failed");
    return EPHW_ENOMEM;
  }
  s->stage_bytes = bytes;
  return EPHW_OK;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device buffers of one call.  `act`, `seg` and `probs` come first and in this
// order: one copy from the pinned staging fills all three.
struct PairWs {
  int32_t* act = nullptr;    // [na] index of each group that owns a pair (q or k)
  int64_t* seg = nullptr;    // [na + 1] pair offsets of those groups
  GroupProblem* probs = nullptr;  // [na]
  int32_t* pair_idx = nullptr;    // [npairs] the group index of every pair (q by q, k by k)
  double* qa = nullptr;      // by q: [na][3] coordinates of the active q
  void* pq = nullptr;        // T [nqp][np]: Rp phases of the q the call needs
  double *pqc = nullptr, *lam = nullptr, *e = nullptr, *hk = nullptr, *jwork = nullptr;
  void* u = nullptr;         // T [nqp][nm][nm]
  void* first = nullptr;     // by q: g(Re,q) of a batch; by k: P_k rows of a chunk
  void* big = nullptr;       // by q: G_nu [Ne][qb E]; by k: G'(k,Rp) [kb][Np][E]
  void* pg = nullptr;        // gathered phase rows of the pairs of a group chunk
  void* wc = nullptr;        // [pairs][E] second-stage sums
  void* wnu = nullptr;       // by k: [pairs][E] after the mode vectors
  double* loss = nullptr;    // [pairs]
  int* queues = nullptr;     // [chunks][kGroupQueues]
  size_t bytes = 0;
};

struct PairPlan {
  bool by_k = false;
  int64_t na = 0, npairs = 0, nqp = 0;      // groups owning pairs, pairs, q points with phases
  int64_t chunk = 0, nchunk = 0, max_pairs = 0;
  size_t first_bytes = 0, big_bytes = 0, pg_row = 0;
};

PairWs pair_layout(const ephw_system* s, int kind, const PairPlan& pl, char* base) {
  PairWs w;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += al256(bytes);
    return p;
  };
  const size_t cs = csize(kind);
  const int64_t nm = s->nm, E = nm * (int64_t)s->nw * s->nw;
  w.act = reinterpret_cast<int32_t*>(take((size_t)pl.na * 4));
  w.seg = reinterpret_cast<int64_t*>(take((size_t)(pl.na + 1) * 8));
  w.probs = reinterpret_cast<GroupProblem*>(take((size_t)pl.na * sizeof(GroupProblem)));
  w.pair_idx = reinterpret_cast<int32_t*>(take((size_t)pl.npairs * 4));
  if (!pl.by_k) w.qa = reinterpret_cast<double*>(take((size_t)pl.na * 24));
  w.pq = take((size_t)pl.nqp * s->np * cs);
  w.pqc = reinterpret_cast<double*>(take((size_t)pl.nqp * s->nc * 16));
  w.lam = reinterpret_cast<double*>(take((size_t)pl.nqp * nm * 8));
  w.e = reinterpret_cast<double*>(take((size_t)pl.nqp * nm * nm * 16));
  w.hk = reinterpret_cast<double*>(take((size_t)pl.nqp * nm * nm * 16));
  const int64_t jw = jacobi_work_doubles((int)nm, pl.nqp);
  if (jw > 0) w.jwork = reinterpret_cast<double*>(take((size_t)jw * 8));
  w.u = take((size_t)pl.nqp * nm * nm * cs);
  w.first = take(pl.first_bytes);
  w.big = take(pl.big_bytes);
  w.pg = take((size_t)pl.max_pairs * pl.pg_row * cs);
  w.wc = take((size_t)pl.max_pairs * E * cs);
  if (pl.by_k) w.wnu = take((size_t)pl.max_pairs * E * cs);
  w.loss = reinterpret_cast<double*>(take((size_t)pl.max_pairs * 8));
  w.queues = reinterpret_cast<int*>(take((size_t)pl.nchunk * kGroupQueues * sizeof(int)));
  w.bytes = off;
  return w;
}

}  // namespace
}  // namespace ephw

using namespace ephw;

extern "C" {

ephw_status ephw_interpolate_pairs(ephw_kset* ks, const double* q, int64_t nq, int32_t order,
                                   const int64_t* pair_start, const int32_t* pair_other, const int32_t* pair_kq,
                                   int64_t q_offset, int32_t prec, uint32_t flags, int32_t band_lo,
                                   int32_t band_count, void* g_out, double* band_sum, double* loss,
                                   uint64_t loss_seed, void* stream) {
  if (!ks || nq < 0 || (nq > 0 && (!q || !pair_start)) || q_offset < 0 ||
      (order != EPHW_PAIRS_BY_Q && order != EPHW_PAIRS_BY_K)) {
    set_error("ephw_interpolate_pairs: invalid argument");
    return EPHW_EINVAL;
  }
  if (prec != ks->prec) {
    set_error("ephw_interpolate_pairs: precision differs from the k-set's");
    return EPHW_EINVAL;
  }
  const uint32_t known = EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS | EPHW_OUT_WANNIER;
  if ((flags & ~known) || !(flags & (EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS)) ||
      ((flags & EPHW_OUT_WANNIER) && (flags & EPHW_OUT_LOSS))) {
    set_error("ephw_interpolate_pairs: flags must request g, band sums or the loss (no loss in the Wannier gauge)");
    return EPHW_EINVAL;
  }
  if (band_count < 0 || (band_count > 0 && (band_lo < 0 || band_lo + band_count > ks->sys->nw ||
                                            (flags & EPHW_OUT_WANNIER)))) {
    set_error("ephw_interpolate_pairs: the band window needs 0 <= band_lo, band_lo + band_count <= nw, "
              "and rotated output");
    return EPHW_EINVAL;
  }
  if (nq == 0 || ks->nk == 0) return EPHW_OK;
  const bool by_k = order == EPHW_PAIRS_BY_K;
  const int64_t nmajor = by_k ? ks->nk : nq;
  if (pair_start[0] != 0) {
    set_error("ephw_interpolate_pairs: pair_start[0] must be 0");
    return EPHW_EINVAL;
  }
  std::vector<int32_t> act;
  for (int64_t i = 0; i < nmajor; ++i) {
    if (pair_start[i + 1] < pair_start[i]) {
      set_error("ephw_interpolate_pairs: pair_start must not decrease");
      return EPHW_EINVAL;
    }
    if (pair_start[i + 1] > pair_start[i]) act.push_back((int32_t)i);
  }
  const int64_t npairs = pair_start[nmajor];
  if (npairs == 0) return EPHW_OK;
  if (!pair_other || !pair_kq || ((flags & EPHW_OUT_G) && !g_out) || ((flags & EPHW_OUT_BAND_SUM) && !band_sum) ||
      ((flags & EPHW_OUT_LOSS) && !loss)) {
    set_error("ephw_interpolate_pairs: a required buffer is NULL");
    return EPHW_EINVAL;
  }
  ephw_system* s = ks->sys;
  if (s->nw > 32) {
    set_error("ephw_interpolate_pairs: systems with more than 32 bands are not supported");
    return EPHW_EUNSUPPORTED;
  }
  if (prec == EPHW_FP32_COMP) {
    set_error("ephw_interpolate_pairs: FP64 or FP32 k-sets only");
    return EPHW_EUNSUPPORTED;
  }
  if (nq > 0x7fffffff || ks->nk > 0x7fffffff || npairs > 0x7fffffff) {
    set_error("ephw_interpolate_pairs: more than 2^31 points or pairs");
    return EPHW_EUNSUPPORTED;
  }
  hipStream_t st = as_stream(stream);
  const int kind = prec_kind(prec);
  const size_t cs = csize(kind);
  const bool wannier = (flags & EPHW_OUT_WANNIER) != 0;
  const int nw = s->nw, nm = s->nm;
  const int64_t nw2 = (int64_t)nw * nw, E = nm * nw2, ne = s->ne, np = s->np;

  // plan: groups of active q (by q) or chunks of active k (by k) such that the
  // chunk's buffers stay within 8 GB; by q at most 128 q per batch (the
  // Eq. (9) GEMM's tile height)
  PairPlan pl;
  pl.by_k = by_k;
  pl.na = (int64_t)act.size();
  pl.npairs = npairs;
  pl.nqp = by_k ? nq : pl.na;
  pl.pg_row = by_k ? (size_t)np : (size_t)ne;
  std::vector<int64_t> seg(pl.na + 1);
  for (int64_t i = 0; i < pl.na; ++i) seg[i] = pair_start[act[i]];
  seg[pl.na] = npairs;
  const double budget = 8.0 * 1024 * 1024 * 1024;
  auto plan_bytes = [&](int64_t c, int64_t* most) {
    int64_t m = 0;
    for (int64_t a0 = 0; a0 < pl.na; a0 += c) m = std::max(m, seg[std::min(pl.na, a0 + c)] - seg[a0]);
    *most = m;
    const double fixed = by_k ? (double)c * (double)(ne + np * E) : 2.0 * (double)c * (double)ne * (double)E;
    return (double)cs * (fixed + (double)m * (double)(pl.pg_row + (by_k ? 2 : 1) * E));
  };
  int64_t chunk = by_k ? pl.na : std::min<int64_t>(pl.na, s->q_batch > 0 ? s->q_batch : 128);
  int64_t most = 0;
  while (chunk > 1 && plan_bytes(chunk, &most) > budget) chunk = (chunk + 1) / 2;
  plan_bytes(chunk, &most);
  pl.chunk = chunk;
  pl.nchunk = ceil_div(pl.na, chunk);
  pl.max_pairs = most;
  pl.first_bytes = by_k ? (size_t)chunk * ne * cs : (size_t)chunk * ne * E * cs;
  pl.big_bytes = by_k ? (size_t)chunk * np * E * cs : (size_t)chunk * ne * E * cs;
  const int64_t lda_pair = by_k ? np : ne, ldb_pair = by_k ? E : chunk * E;
  if (!cgemm_grouped_fits(kind, lda_pair, ldb_pair)) {
    set_error("ephw_interpolate_pairs: leading dimensions too large for the grouped GEMM");
    return EPHW_EUNSUPPORTED;
  }

  const size_t need = pair_layout(s, kind, pl, nullptr).bytes;
  EPHW_TRY(ws_need(s, WS_PAIRSET, need));
  const PairWs w = pair_layout(s, kind, pl, static_cast<char*>(wsp(s, WS_PAIRSET)));

  // one grouped-GEMM problem per group: by q, W_q = P_k[kept k] G_nu(q); by
  // k, W_k = P_q[kept q] G'(k); operand pointers relative to the chunk's buffers
  const int cfg = 1;   // 64 x 64 tiles: the problems have tens of rows
  std::vector<GroupProblem> probs(pl.na);
  std::vector<int64_t> chunk_tiles(pl.nchunk);
  for (int64_t c = 0; c < pl.nchunk; ++c) {
    const int64_t a0 = c * chunk, a1 = std::min(pl.na, a0 + chunk), nb = a1 - a0;
    for (int64_t i = a0; i < a1; ++i) {
      GroupProblem& P = probs[i];
      P.M = seg[i + 1] - seg[i];
      P.N = E;
      P.K = by_k ? np : ne;
      P.A = static_cast<const char*>(w.pg) + (size_t)(seg[i] - seg[a0]) * pl.pg_row * cs;
      P.lda = lda_pair;
      P.B = by_k ? static_cast<const char*>(w.big) + (size_t)(i - a0) * np * E * cs
                 : static_cast<const char*>(w.big) + (size_t)(i - a0) * E * cs;
      P.ldb = by_k ? E : nb * E;
      P.C = static_cast<char*>(w.wc) + (size_t)(seg[i] - seg[a0]) * E * cs;
      P.ldc = E;
      P.cfg = cfg;
    }
    chunk_tiles[c] = cgemm_grouped_layout(kind, probs.data() + a0, (int)nb);
  }
  {
    const size_t b_a = (size_t)pl.na * 4, b_s = (size_t)(pl.na + 1) * 8, b_p = (size_t)pl.na * sizeof(GroupProblem);
    const size_t o_s = al256(b_a), o_p = o_s + al256(b_s), total = o_p + b_p;
    EPHW_TRY(stage_reserve(s, total));
    char* h = static_cast<char*>(s->stage_host);
    memcpy(h, act.data(), b_a);
    memcpy(h + o_s, seg.data(), b_s);
    memcpy(h + o_p, probs.data(), b_p);
    EPHW_HIP(hipMemcpyAsync(w.act, h, total, hipMemcpyHostToDevice, st));
    EPHW_HIP(hipEventRecord(s->staged, st));
  }
  EPHW_TRY(cgemm_grouped_reset(w.queues, (int)(pl.nchunk * kGroupQueues), st));

  // the q side: Rp phases, D(q) eigensolves and mode vectors of the q that own
  // pairs (by q) or of every q of the list (by k); the group index of every pair
  const double* qp = q;
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    hipLaunchKernelGGL(fill_segments_kernel, dim3((unsigned)pl.na), dim3(256), 0, st, w.seg, w.act, w.pair_idx);
    EPHW_CHECK_LAUNCH();
    if (!by_k) {
      hipLaunchKernelGGL(gather_q_kernel, dim3((unsigned)ceil_div(3 * pl.na, 256)), dim3(256), 0, st, q, w.act,
                         pl.na, w.qa);
      EPHW_CHECK_LAUNCH();
      qp = w.qa;
    }
    EPHW_TRY(phase_matrix(kind, qp, pl.nqp, s->r_p, s->w_p, s->np, w.pq, st));
    EPHW_TRY(phase_matrix(0, qp, pl.nqp, s->r_c, s->w_c, s->nc, w.pqc, st));
  }
  EPHW_TRY(interp_eigh_ws(s, w.pqc, pl.nqp, s->nc, s->c_scaled, nm, w.lam, w.e, w.hk, w.jwork, true, st));
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st);
    EPHW_TRY(mode_vectors(kind, w.e, pl.nqp, nm, s->ism, w.u, st));
  }

  int grid = 0;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->ctx->device) != hipSuccess || cus <= 0)
      cus = 256;
    grid = cus * cgemm_grouped_blocks_per_cu(kind, cfg);
  }
  auto gather = [&](const void* src, int64_t nsrc, const int32_t* idx, int64_t cnt, int64_t width, void* dst) {
    return kind == 0 ? gather_complex_rows<double>(src, nsrc, idx, cnt, width, dst, s->ctx->status, st)
                     : gather_complex_rows<float>(src, nsrc, idx, cnt, width, dst, s->ctx->status, st);
  };
  for (int64_t c = 0; c < pl.nchunk; ++c) {
    const int64_t a0 = c * chunk, a1 = std::min(pl.na, a0 + chunk), nb = a1 - a0;
    const int64_t p0 = seg[a0], nbp = seg[a1] - p0;
    const void* wpair = w.wc;   // per-pair sums the band rotations read
    if (!by_k) {
      // Eq. (9) for the batch's q, mode vectors, then the Re sum per q
      GemmParams rp;
      rp.M = nb;
      rp.N = ne * E;
      rp.K = np;
      rp.A = static_cast<const char*>(w.pq) + (size_t)a0 * np * cs;
      rp.lda = np;
      rp.B = s->g;
      rp.ldb = rp.N;
      rp.C = w.first;
      rp.ldc = rp.N;
      {
        Stage sg_(s, EPHW_STAGE_RP_GEMM, st);
        EPHW_TRY(cgemm(kind, rp, st));
      }
      {
        Stage sg_(s, EPHW_STAGE_MODE_ROT, st);
        EPHW_TRY(mode_rotate(kind, w.first,
                             wannier ? nullptr : static_cast<const char*>(w.u) + (size_t)a0 * nm * nm * cs, w.big, ne,
                             (int)nb, nm, nw2, st));
      }
      Stage sg_(s, EPHW_STAGE_RE_GEMM, st);
      EPHW_TRY(gather(ks->pk, ks->nk, pair_other + p0, nbp, ne, w.pg));
      EPHW_TRY(cgemm_grouped(kind, cfg, w.probs + a0, (int)nb, chunk_tiles[c],
                             (int)std::min<int64_t>(grid, chunk_tiles[c]), w.queues + c * kGroupQueues, st));
    } else {
      // the Re sum over every Rp for the chunk's k: one GEMM batched over Rp,
      // G'[k][Rp][:] = P_k[k][:] g(Rp)[Re][:]
      {
        Stage sg_(s, EPHW_STAGE_RE_GEMM, st);
        EPHW_TRY(gather(ks->pk, ks->nk, w.act + a0, nb, ne, w.first));
        GemmParams re;
        re.M = nb;
        re.N = E;
        re.K = ne;
        re.batch = np;
        re.A = w.first;
        re.lda = ne;
        re.strideA = 0;
        re.B = s->g;
        re.ldb = E;
        re.strideB = ne * E;
        re.C = w.big;
        re.ldc = np * E;
        re.strideC = E;
        EPHW_TRY(cgemm(kind, re, st));
      }
      // the Rp sum per k over its kept q, then the mode vectors per pair
      {
        Stage sg_(s, EPHW_STAGE_RP_GEMM, st);
        EPHW_TRY(gather(w.pq, nq, pair_other + p0, nbp, np, w.pg));
        EPHW_TRY(cgemm_grouped(kind, cfg, w.probs + a0, (int)nb, chunk_tiles[c],
                               (int)std::min<int64_t>(grid, chunk_tiles[c]), w.queues + c * kGroupQueues, st));
      }
      if (!wannier) {
        Stage sg_(s, EPHW_STAGE_MODE_ROT, st);
        const int64_t n = nbp * nw2;
        if (kind == 0)
          hipLaunchKernelGGL(pair_mode_rotate_kernel<double>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st,
                             static_cast<const double*>(w.wc), static_cast<const double*>(w.u), pair_other + p0, nq,
                             nbp, nm, (int)nw2, static_cast<double*>(w.wnu), s->ctx->status);
        else
          hipLaunchKernelGGL(pair_mode_rotate_kernel<float>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st,
                             static_cast<const float*>(w.wc), static_cast<const float*>(w.u), pair_other + p0, nq,
                             nbp, nm, (int)nw2, static_cast<float*>(w.wnu), s->ctx->status);
        EPHW_CHECK_LAUNCH();
        wpair = w.wnu;
      }
    }
    // band rotations and epilogues per pair
    BandRotateArgs br;
    br.W = wpair;
    br.Vk = wannier ? nullptr : ks->vt;
    br.Vkq = nullptr;
    br.kq_index = pair_kq + p0;
    br.nk = nbp;
    br.k0 = 0;
    br.nk_tile = nbp;
    br.qb = 1;
    br.nm = nm;
    br.nw = nw;
    br.flags = flags;
    const int64_t nbo = band_count > 0 ? band_count : nw, Eo = nm * nbo * nbo;
    br.g_out = (flags & EPHW_OUT_G) ? static_cast<char*>(g_out) + (size_t)p0 * Eo * cs : nullptr;
    br.band_lo = band_lo;
    br.band_n = band_count;
    br.band_sum = (flags & EPHW_OUT_BAND_SUM) ? band_sum + p0 * nm : nullptr;
    br.loss_partial = w.loss;
    br.loss_seed = loss_seed;
    br.q_global0 = q_offset;
    br.status = s->ctx->status;
    br.pair_k = by_k ? w.pair_idx + p0 : pair_other + p0;
    br.pair_q = by_k ? pair_other + p0 : w.pair_idx + p0;
    br.nk_set = ks->nk;
    {
      Stage sg_(s, EPHW_STAGE_BAND_ROT, st);
      EPHW_TRY(band_rotate(kind, br, st));
    }
    if (flags & EPHW_OUT_LOSS) {
      Stage sg_(s, EPHW_STAGE_OTHER, st);
      EPHW_TRY(sum_into(w.loss, nbp, loss, st));
    }
  }
  return EPHW_OK;
}

}  // extern "C"
