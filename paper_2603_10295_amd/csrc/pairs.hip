// Eq. (7) on an explicit list of (k, q) pairs: the pairs that survive the
// energy-window pre-screening the paper applies before interpolating.
//
// The q side is that of ephw_interpolate (Eq. (9) as one GEMM per batch of q,
// mode vectors applied to g(Re,q)), restricted to the q that own a pair.  The
// Re sum of Eq. (10) then runs on the kept pairs only: per q, the phase rows
// P_k of its kept k are gathered into a contiguous block, and
//   W_q[kept k][nu m' n'] = P_k[kept k][Re] G_nu(Re, q)
// is one problem of a grouped GEMM (all q of a batch in one persistent
// launch; the problems have as many rows as the q has kept pairs).  The band
// rotations V(k+q)^dagger W V(k) and the epilogues run per pair in the
// band-rotation kernel's pair mode.  Outputs are indexed by pair.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace ephw {
namespace {

// dst[i][:] = src[idx[i]][:] for complex rows of `width` values
template <typename T>
__global__ void gather_complex_rows_kernel(const T* __restrict__ src, int64_t nsrc, const int32_t* __restrict__ idx,
                                           int64_t cnt, int64_t width, T* __restrict__ dst, uint32_t* status) {
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

// pair_q[p] = q for the pairs of active q number i: [seg[i], seg[i+1])
__global__ void fill_pair_q_kernel(const int64_t* __restrict__ seg, const int32_t* __restrict__ qidx,
                                   int32_t* __restrict__ pair_q) {
  const int64_t i = blockIdx.x;
  const int32_t q = qidx[i];
  for (int64_t p = seg[i] + threadIdx.x; p < seg[i + 1]; p += blockDim.x) pair_q[p] = q;
}

__global__ void gather_q_kernel(const double* __restrict__ q, const int32_t* __restrict__ qidx, int64_t n,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * n) out[i] = q[3 * (int64_t)qidx[i / 3] + i % 3];
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

struct PairWs {
  int32_t* qidx = nullptr;   // [nqa] original index of each active q
  int64_t* seg = nullptr;    // [nqa + 1] pair offsets of the active q
  int32_t* pair_q = nullptr; // [npairs]
  double* qa = nullptr;      // [nqa][3]
  void* pq = nullptr;        // T [nqa][np]
  double *pqc = nullptr, *lam = nullptr, *e = nullptr, *hk = nullptr, *jwork = nullptr;
  void* u = nullptr;         // T [nqa][nm][nm]
  void *g = nullptr, *gnu = nullptr, *pg = nullptr, *wc = nullptr;
  double* loss = nullptr;    // [max pairs of a batch]
  GroupProblem* probs = nullptr;  // [nqa]
  int* queues = nullptr;     // [batches][kGroupQueues]
  size_t bytes = 0;
};

PairWs pair_layout(const ephw_system* s, int kind, int64_t nqa, int64_t npairs, int64_t qb, int64_t max_pairs,
                   int64_t nbatch, char* base) {
  PairWs w;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const size_t cs = csize(kind);
  const int64_t nm = s->nm, E = nm * (int64_t)s->nw * s->nw;
  // qidx, seg and probs first and in this order: one copy fills all three
  w.qidx = reinterpret_cast<int32_t*>(take((size_t)nqa * 4));
  w.seg = reinterpret_cast<int64_t*>(take((size_t)(nqa + 1) * 8));
  w.probs = reinterpret_cast<GroupProblem*>(take((size_t)nqa * sizeof(GroupProblem)));
  w.pair_q = reinterpret_cast<int32_t*>(take((size_t)npairs * 4));
  w.qa = reinterpret_cast<double*>(take((size_t)nqa * 24));
  w.pq = take((size_t)nqa * s->np * cs);
  w.pqc = reinterpret_cast<double*>(take((size_t)nqa * s->nc * 16));
  w.lam = reinterpret_cast<double*>(take((size_t)nqa * nm * 8));
  w.e = reinterpret_cast<double*>(take((size_t)nqa * nm * nm * 16));
  w.hk = reinterpret_cast<double*>(take((size_t)nqa * nm * nm * 16));
  const int64_t jw = jacobi_work_doubles((int)nm, nqa);
  if (jw > 0) w.jwork = reinterpret_cast<double*>(take((size_t)jw * 8));
  w.u = take((size_t)nqa * nm * nm * cs);
  w.g = take((size_t)qb * s->ne * E * cs);
  w.gnu = take((size_t)qb * s->ne * E * cs);
  w.pg = take((size_t)max_pairs * s->ne * cs);
  w.wc = take((size_t)max_pairs * E * cs);
  w.loss = reinterpret_cast<double*>(take((size_t)max_pairs * 8));
  w.queues = reinterpret_cast<int*>(take((size_t)nbatch * kGroupQueues * sizeof(int)));
  w.bytes = off;
  return w;
}

}  // namespace
}  // namespace ephw

using namespace ephw;

extern "C" {

ephw_status ephw_interpolate_pairs(ephw_kset* ks, const double* q, int64_t nq, const int64_t* pair_start,
                                   const int32_t* pair_k, const int32_t* pair_kq, int64_t q_offset, int32_t prec,
                                   uint32_t flags, void* g_out, double* band_sum, double* loss, uint64_t loss_seed,
                                   void* stream) {
  if (!ks || nq < 0 || (nq > 0 && (!q || !pair_start)) || q_offset < 0) {
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
  if (nq == 0) return EPHW_OK;
  if (pair_start[0] != 0) {
    set_error("ephw_interpolate_pairs: pair_start[0] must be 0");
    return EPHW_EINVAL;
  }
  std::vector<int32_t> act;
  for (int64_t i = 0; i < nq; ++i) {
    if (pair_start[i + 1] < pair_start[i]) {
      set_error("ephw_interpolate_pairs: pair_start must not decrease");
      return EPHW_EINVAL;
    }
    if (pair_start[i + 1] > pair_start[i]) act.push_back((int32_t)i);
  }
  const int64_t npairs = pair_start[nq];
  if (npairs == 0) return EPHW_OK;
  if (!pair_k || !pair_kq || ((flags & EPHW_OUT_G) && !g_out) || ((flags & EPHW_OUT_BAND_SUM) && !band_sum) ||
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
  if (nq > 0x7fffffff || ks->nk > 0x7fffffff) {
    set_error("ephw_interpolate_pairs: more than 2^31 points");
    return EPHW_EUNSUPPORTED;
  }
  hipStream_t st = as_stream(stream);
  const int kind = prec_kind(prec);
  const size_t cs = csize(kind);
  const bool wannier = (flags & EPHW_OUT_WANNIER) != 0;
  const int nw = s->nw, nm = s->nm;
  const int64_t nw2 = (int64_t)nw * nw, E = nm * nw2, ne = s->ne;
  const int64_t nqa = (int64_t)act.size();

  // q batches: up to 128 active q, within 8 GB for the two g(Re,q) sweeps and
  // the gathered phase rows and Re-sum outputs of the batch's pairs
  int64_t qb = s->q_batch > 0 ? s->q_batch : 128;
  auto batch_bytes = [&](int64_t b) {
    int64_t most = 0;
    for (int64_t a0 = 0; a0 < nqa; a0 += b) {
      const int64_t a1 = std::min(nqa, a0 + b);
      most = std::max(most, pair_start[act[a1 - 1] + 1] - pair_start[act[a0]]);
    }
    return std::make_pair((double)cs * (2.0 * b * ne * E + (double)most * (ne + E)), most);
  };
  while (qb > 1 && batch_bytes(qb).first > 8.0 * 1024 * 1024 * 1024) qb /= 2;
  if (qb > nqa) qb = nqa;
  const int64_t max_pairs = batch_bytes(qb).second;
  const int64_t nbatch = ceil_div(nqa, qb);
  if (!cgemm_grouped_fits(kind, ne, qb * E) || !cgemm_grouped_fits(kind, ne, E)) {
    set_error("ephw_interpolate_pairs: leading dimensions too large for the grouped GEMM");
    return EPHW_EUNSUPPORTED;
  }

  const size_t need = pair_layout(s, kind, nqa, npairs, qb, max_pairs, nbatch, nullptr).bytes;
  EPHW_TRY(ws_need(s, WS_PAIRSET, need));
  const PairWs w = pair_layout(s, kind, nqa, npairs, qb, max_pairs, nbatch, static_cast<char*>(wsp(s, WS_PAIRSET)));

  // per active q: its index, its pair range; one grouped-GEMM problem per q,
  // laid out per batch (operand pointers relative to the batch's buffers)
  std::vector<int64_t> seg(nqa + 1);
  for (int64_t i = 0; i < nqa; ++i) seg[i] = pair_start[act[i]];
  seg[nqa] = npairs;
  const int cfg = 1;   // 64 x 64 tiles: the problems have tens of rows
  std::vector<GroupProblem> probs(nqa);
  std::vector<int64_t> batch_tiles(nbatch);
  for (int64_t b = 0; b < nbatch; ++b) {
    const int64_t a0 = b * qb, a1 = std::min(nqa, a0 + qb), nb = a1 - a0;
    for (int64_t i = a0; i < a1; ++i) {
      GroupProblem& P = probs[i];
      P.M = seg[i + 1] - seg[i];
      P.N = E;
      P.K = ne;
      P.A = static_cast<const char*>(w.pg) + (size_t)(seg[i] - seg[a0]) * ne * cs;
      P.lda = ne;
      P.B = static_cast<const char*>(w.gnu) + (size_t)(i - a0) * E * cs;
      P.ldb = nb * E;
      P.C = static_cast<char*>(w.wc) + (size_t)(seg[i] - seg[a0]) * E * cs;
      P.ldc = E;
      P.cfg = cfg;
    }
    batch_tiles[b] = cgemm_grouped_layout(kind, probs.data() + a0, (int)nb);
  }
  {
    // one pinned staging block, copied once: q indices, pair offsets, problems
    const size_t b_q = (size_t)nqa * 4, b_s = (size_t)(nqa + 1) * 8, b_p = (size_t)nqa * sizeof(GroupProblem);
    const size_t o_s = (b_q + 255) & ~(size_t)255, o_p = o_s + ((b_s + 255) & ~(size_t)255), total = o_p + b_p;
    EPHW_TRY(stage_reserve(s, total));
    char* h = static_cast<char*>(s->stage_host);
    memcpy(h, act.data(), b_q);
    memcpy(h + o_s, seg.data(), b_s);
    memcpy(h + o_p, probs.data(), b_p);
    // the three device arrays are consecutive in the workspace with the same offsets
    EPHW_HIP(hipMemcpyAsync(w.qidx, h, total, hipMemcpyHostToDevice, st));
    EPHW_HIP(hipEventRecord(s->staged, st));
  }
  EPHW_TRY(cgemm_grouped_reset(w.queues, (int)(nbatch * kGroupQueues), st));

  // q side of the active q: coordinates, Rp phases, D(q) eigensolves, mode vectors
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    hipLaunchKernelGGL(gather_q_kernel, dim3((unsigned)ceil_div(3 * nqa, 256)), dim3(256), 0, st, q, w.qidx, nqa,
                       w.qa);
    EPHW_CHECK_LAUNCH();
    hipLaunchKernelGGL(fill_pair_q_kernel, dim3((unsigned)nqa), dim3(256), 0, st, w.seg, w.qidx, w.pair_q);
    EPHW_CHECK_LAUNCH();
    EPHW_TRY(phase_matrix(kind, w.qa, nqa, s->r_p, s->w_p, s->np, w.pq, st));
    EPHW_TRY(phase_matrix(0, w.qa, nqa, s->r_c, s->w_c, s->nc, w.pqc, st));
  }
  EPHW_TRY(interp_eigh_ws(s, w.pqc, nqa, s->nc, s->c_scaled, nm, w.lam, w.e, w.hk, w.jwork, true, st));
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st);
    EPHW_TRY(mode_vectors(kind, w.e, nqa, nm, s->ism, w.u, st));
  }

  int grid = 0;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->ctx->device) != hipSuccess || cus <= 0)
      cus = 256;
    grid = cus * cgemm_grouped_blocks_per_cu(kind, cfg);
  }
  for (int64_t b = 0; b < nbatch; ++b) {
    const int64_t a0 = b * qb, a1 = std::min(nqa, a0 + qb), nb = a1 - a0;
    const int64_t p0 = seg[a0], nbp = seg[a1] - p0;
    // Eq. (9) for the batch's q
    GemmParams rp;
    rp.M = nb;
    rp.N = ne * E;
    rp.K = s->np;
    rp.A = static_cast<const char*>(w.pq) + (size_t)a0 * s->np * cs;
    rp.lda = s->np;
    rp.B = s->g;
    rp.ldb = rp.N;
    rp.C = w.g;
    rp.ldc = rp.N;
    {
      Stage sg_(s, EPHW_STAGE_RP_GEMM, st);
      EPHW_TRY(cgemm(kind, rp, st));
    }
    {
      Stage sg_(s, EPHW_STAGE_MODE_ROT, st);
      EPHW_TRY(mode_rotate(kind, w.g, wannier ? nullptr : static_cast<const char*>(w.u) + (size_t)a0 * nm * nm * cs,
                           w.gnu, ne, (int)nb, nm, nw2, st));
    }
    // Eq. (10), Re part, on the kept pairs: gathered P_k rows, one problem per q
    {
      Stage sg_(s, EPHW_STAGE_RE_GEMM, st);
      const dim3 gg((unsigned)std::min<int64_t>(ceil_div(ne, 256), 64));
      for (int64_t c0 = 0; c0 < nbp; c0 += 65535) {
        const int64_t cn = std::min<int64_t>(65535, nbp - c0);
        if (kind == 0)
          hipLaunchKernelGGL(gather_complex_rows_kernel<double>, dim3(gg.x, (unsigned)cn), dim3(256), 0, st,
                             static_cast<const double*>(ks->pk), ks->nk, pair_k + p0 + c0, cn, ne,
                             static_cast<double*>(w.pg) + 2 * c0 * ne, s->ctx->status);
        else
          hipLaunchKernelGGL(gather_complex_rows_kernel<float>, dim3(gg.x, (unsigned)cn), dim3(256), 0, st,
                             static_cast<const float*>(ks->pk), ks->nk, pair_k + p0 + c0, cn, ne,
                             static_cast<float*>(w.pg) + 2 * c0 * ne, s->ctx->status);
        EPHW_CHECK_LAUNCH();
      }
      EPHW_TRY(cgemm_grouped(kind, cfg, w.probs + a0, (int)nb, batch_tiles[b],
                             (int)std::min<int64_t>(grid, batch_tiles[b]), w.queues + b * kGroupQueues, st));
    }
    // band rotations and epilogues per pair
    BandRotateArgs br;
    br.W = w.wc;
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
    br.g_out = (flags & EPHW_OUT_G) ? static_cast<char*>(g_out) + (size_t)p0 * E * cs : nullptr;
    br.band_sum = (flags & EPHW_OUT_BAND_SUM) ? band_sum + p0 * nm : nullptr;
    br.loss_partial = w.loss;
    br.loss_seed = loss_seed;
    br.q_global0 = q_offset;
    br.status = s->ctx->status;
    br.pair_k = pair_k + p0;
    br.pair_q = w.pair_q + p0;
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
