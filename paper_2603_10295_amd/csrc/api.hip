// Host side of the libephw C ABI: validation, ownership, workspaces and the
// sequencing of the interpolation (Eqs. (7), (9), (10)) on a HIP stream.
#include <math.h>

#include <cmath>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace ephw {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

ephw_status interp_eigh_ws(ephw_system* s, const double* phase, int64_t n, int64_t nr, const double* mats, int dim,
                           double* out_eps, double* out_v, double* hk, double* jwork, bool stages, hipStream_t st) {
  const int64_t d2 = (int64_t)dim * dim;
  Stage sg_(s, EPHW_STAGE_EIG, st, stages);
  GemmParams p;
  p.M = n;
  p.N = d2;
  p.K = nr;
  p.A = phase;
  p.lda = nr;
  p.B = mats;
  p.ldb = d2;
  p.C = hk;
  p.ldc = d2;
  EPHW_TRY(cgemm(0, p, st));
  return jacobi_eigh(hk, n, dim, out_eps, out_v, jwork, s->ctx->status, st);
}

}  // namespace ephw

namespace {

ephw_status interp_eigh(ephw_system* s, const double* phase, int64_t n, int64_t nr, const double* mats,
                        int dim, double* out_eps, double* out_v, hipStream_t st) {
  const int64_t d2 = (int64_t)dim * dim;
  EPHW_TRY(ws_need(s, WS_HK, (size_t)n * d2 * 16));
  const int64_t jw = jacobi_work_doubles(dim, n);
  if (jw > 0) EPHW_TRY(ws_need(s, WS_JWORK, (size_t)jw * 8));
  return interp_eigh_ws(s, phase, n, nr, mats, dim, out_eps, out_v, static_cast<double*>(wsp(s, WS_HK)),
                        jw > 0 ? static_cast<double*>(wsp(s, WS_JWORK)) : nullptr, true, st);
}

int32_t pick_q_batch(const ephw_system* s, int64_t nk, int64_t nq, int kind) {
  if (s->q_batch > 0) return (int32_t)(s->q_batch < nq ? s->q_batch : nq);
  // q points per sweep: the Rp GEMM has M = q_batch, so a full 128-row tile
  // wants 128; the workspace (Re-GEMM output + two g(Re,q) buffers) is capped
  // at 8 GB of the 288 GB of HBM.
  const int64_t E = (int64_t)s->nm * s->nw * s->nw;
  const double per_q = (double)csize(kind) * E * ((double)nk + 2.0 * (double)s->ne);
  int64_t qb = (int64_t)((8.0 * 1024 * 1024 * 1024) / per_q);
  if (qb >= 128) qb = 128;
  else if (qb >= 64) qb = 64;
  if (qb < 1) qb = 1;
  if (qb > nq) qb = nq;
  return (int32_t)qb;
}

}  // namespace

extern "C" {

const char* ephw_status_string(ephw_status s) {
  switch (s) {
    case EPHW_OK: return "ok";
    case EPHW_EINVAL: return "invalid argument";
    case EPHW_ENOMEM: return "out of device memory";
    case EPHW_EDEVICE: return "HIP runtime error";
    case EPHW_ENOCONV: return "eigensolver did not converge";
    case EPHW_EUNSUPPORTED: return "unsupported request";
    case EPHW_EINDEX: return "k+q index out of range";
    default: return "unknown status";
  }
}

const char* ephw_last_error(void) { return g_last_error.c_str(); }

int32_t ephw_version(void) { return 200; }

ephw_status ephw_ctx_create(int device, ephw_ctx** out) {
  if (!out) {
    set_error("ephw_ctx_create: out is NULL");
    return EPHW_EINVAL;
  }
  *out = nullptr;
  int count = 0;
  EPHW_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) {
    set_error("ephw_ctx_create: no such device");
    return EPHW_EINVAL;
  }
  EPHW_HIP(hipSetDevice(device));
  ephw_ctx* c = new ephw_ctx();
  c->device = device;
  void* p = nullptr;
  ephw_status st = dev_alloc(&p, 2 * sizeof(uint32_t));
  if (st != EPHW_OK) {
    delete c;
    return st;
  }
  c->status = static_cast<uint32_t*>(p);
  const uint32_t init[2] = {0u, (uint32_t)kDefaultSweeps};
  EPHW_HIP(hipMemcpy(c->status, init, sizeof(init), hipMemcpyHostToDevice));
  *out = c;
  return EPHW_OK;
}

ephw_status ephw_ctx_set_limits(ephw_ctx* ctx, int64_t max_device_bytes, int32_t max_sweeps) {
  if (!ctx || max_device_bytes < 0 || max_sweeps < 0 || max_sweeps > kMaxSweepLimit) {
    set_error("ephw_ctx_set_limits: need a context, max_device_bytes >= 0 and 0 <= max_sweeps <= " +
              std::to_string(kMaxSweepLimit));
    return EPHW_EINVAL;
  }
  EPHW_HIP(hipSetDevice(ctx->device));
  EPHW_HIP(hipDeviceSynchronize());   // no kernel of the context reads the limit meanwhile
  const uint32_t sweeps = (uint32_t)max_sweeps;
  EPHW_HIP(hipMemcpy(ctx->status + 1, &sweeps, sizeof(sweeps), hipMemcpyHostToDevice));
  ctx->mem->limit = max_device_bytes;
  return EPHW_OK;
}

ephw_status ephw_ctx_memory(const ephw_ctx* ctx, int64_t* used, int64_t* limit) {
  if (!ctx) {
    set_error("ephw_ctx_memory: ctx is NULL");
    return EPHW_EINVAL;
  }
  if (used) *used = ctx->mem->used.load();
  if (limit) *limit = ctx->mem->limit;
  return EPHW_OK;
}

ephw_status ephw_ctx_destroy(ephw_ctx* ctx) {
  if (!ctx) return EPHW_OK;
  if (ctx->status) (void)hipFree(ctx->status);
  delete ctx;
  return EPHW_OK;
}

ephw_status ephw_ctx_check(ephw_ctx* ctx, void* stream) {
  if (!ctx) {
    set_error("ephw_ctx_check: ctx is NULL");
    return EPHW_EINVAL;
  }
  EPHW_HIP(hipStreamSynchronize(as_stream(stream)));
  uint32_t v = 0;
  EPHW_HIP(hipMemcpy(&v, ctx->status, sizeof(v), hipMemcpyDeviceToHost));
  EPHW_HIP(hipMemset(ctx->status, 0, sizeof(uint32_t)));
  if (v & kStatusIndex) {
    set_error("a k+q index table entry was outside [0, nk)");
    return EPHW_EINDEX;
  }
  if (v & kStatusNoConv) {
    set_error("a Jacobi eigensolve reached its sweep limit");
    return EPHW_ENOCONV;
  }
  return EPHW_OK;
}

ephw_status ephw_system_free(ephw_system* s) {
  if (!s) return EPHW_OK;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {s->r_e, s->r_p, s->r_h, s->r_c, s->w_e, s->w_p, s->w_h, s->w_c,
                  s->h_r, s->c_scaled, s->ism, s->g};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (auto& b : s->ws)
    if (b.p) (void)hipFree(b.p);
  dev_release(s->mem.get(), s->bytes);
  for (auto& r : s->prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : s->prof.pool) (void)hipEventDestroy(e);
  if (s->stage_host) (void)hipHostFree(s->stage_host);
  if (s->staged) (void)hipEventDestroy(s->staged);
  delete s;
  return EPHW_OK;
}

ephw_status ephw_system_load(ephw_ctx* ctx, const ephw_system_desc* d, ephw_system** out) {
  if (!ctx || !d || !out) {
    set_error("ephw_system_load: NULL argument");
    return EPHW_EINVAL;
  }
  *out = nullptr;
  if (d->nw < 1 || d->nw > 256 || d->na < 1 || d->na > 86 || d->ne < 1 || d->np < 1 || d->nh < 1 ||
      d->nc < 1) {
    set_error("ephw_system_load: sizes out of range (1<=nw<=256, 1<=na<=86, counts >= 1)");
    return EPHW_EINVAL;
  }
  if (!d->r_e || !d->r_p || !d->r_h || !d->r_c || !d->h_r || !d->c_r || !d->mass) {
    set_error("ephw_system_load: a required array is NULL");
    return EPHW_EINVAL;
  }
  if (d->g_dtype != EPHW_C128 && d->g_dtype != EPHW_C64) {
    set_error("ephw_system_load: g_dtype must be EPHW_C128 or EPHW_C64");
    return EPHW_EINVAL;
  }
  for (int a = 0; a < d->na; ++a)
    if (!(d->mass[a] > 0.0)) {
      set_error("ephw_system_load: masses must be positive");
      return EPHW_EINVAL;
    }
  EPHW_HIP(hipSetDevice(ctx->device));
  ephw_system* s = new ephw_system();
  s->ctx = ctx;
  s->mem = ctx->mem;
  s->nw = d->nw;
  s->na = d->na;
  s->nm = 3 * d->na;
  s->ne = d->ne;
  s->np = d->np;
  s->nh = d->nh;
  s->nc = d->nc;
  s->g_kind = d->g_dtype == EPHW_C128 ? 0 : 1;
  const int nm = s->nm;
  ephw_status st = EPHW_OK;
  auto fail = [&](ephw_status e) {
    ephw_system_free(s);
    return e;
  };
  if ((st = upload(&s->r_e, d->r_e, 3 * d->ne, &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
  if ((st = upload(&s->r_p, d->r_p, 3 * d->np, &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
  if ((st = upload(&s->r_h, d->r_h, 3 * d->nh, &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
  if ((st = upload(&s->r_c, d->r_c, 3 * d->nc, &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
  auto weights = [&](double** dst, const double* w, int64_t n) {
    std::vector<double> ones;
    if (!w) {
      ones.assign((size_t)n, 1.0);
      w = ones.data();
    }
    return upload(dst, w, (size_t)n, &s->bytes, s->mem.get());
  };
  if ((st = weights(&s->w_e, d->w_e, d->ne)) != EPHW_OK) return fail(st);
  if ((st = weights(&s->w_p, d->w_p, d->np)) != EPHW_OK) return fail(st);
  if ((st = weights(&s->w_h, d->w_h, d->nh)) != EPHW_OK) return fail(st);
  if ((st = weights(&s->w_c, d->w_c, d->nc)) != EPHW_OK) return fail(st);
  if ((st = upload(&s->h_r, static_cast<const double*>(d->h_r), (size_t)2 * d->nh * d->nw * d->nw,
                   &s->bytes, s->mem.get())) != EPHW_OK)
    return fail(st);
  {
    // C(R) / sqrt(M_kappa M_kappa') as complex128, the B operand of D(q)
    std::vector<double> ism((size_t)nm), cs((size_t)2 * d->nc * nm * nm);
    for (int a = 0; a < nm; ++a) ism[a] = 1.0 / sqrt(d->mass[a / 3]);
    for (int64_t r = 0; r < d->nc; ++r)
      for (int a = 0; a < nm; ++a)
        for (int b = 0; b < nm; ++b) {
          const size_t i = ((size_t)r * nm + a) * nm + b;
          cs[2 * i] = d->c_r[i] * ism[a] * ism[b];
          cs[2 * i + 1] = 0.0;
        }
    if ((st = upload(&s->c_scaled, cs.data(), cs.size(), &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
    if ((st = upload(&s->ism, ism.data(), ism.size(), &s->bytes, s->mem.get())) != EPHW_OK) return fail(st);
  }
  {
    const size_t gbytes = (size_t)d->np * d->ne * nm * d->nw * d->nw * csize(s->g_kind);
    if ((st = dev_alloc(&s->g, gbytes, s->mem.get())) != EPHW_OK) return fail(st);
    s->bytes += (int64_t)gbytes;
    // g NULL: the caller fills it on the device with ephw_system_set_g
    if (d->g && hipMemcpy(s->g, d->g, gbytes, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("ephw_system_load: upload of g failed");
      return fail(EPHW_EDEVICE);
    }
  }
  *out = s;
  return EPHW_OK;
}

ephw_status ephw_system_trim(ephw_system* s) {
  if (!s) {
    set_error("ephw_system_trim: NULL argument");
    return EPHW_EINVAL;
  }
  bool any = false;
  for (auto& b : s->ws) any = any || b.p;
  if (!any) return EPHW_OK;
  EPHW_HIP(hipDeviceSynchronize());
  for (auto& b : s->ws)
    if (b.p) {
      EPHW_HIP(hipFree(b.p));
      s->bytes -= (int64_t)b.bytes;
      dev_release(s->mem.get(), (int64_t)b.bytes);
      b.p = nullptr;
      b.bytes = 0;
    }
  return EPHW_OK;
}

ephw_status ephw_system_set_g(ephw_system* s, const void* g, void* stream) {
  if (!s || !g) {
    set_error("ephw_system_set_g: NULL argument");
    return EPHW_EINVAL;
  }
  const size_t bytes = (size_t)s->np * s->ne * s->nm * s->nw * s->nw * csize(s->g_kind);
  EPHW_HIP(hipMemcpyAsync(s->g, g, bytes, hipMemcpyDeviceToDevice, as_stream(stream)));
  return EPHW_OK;
}

ephw_status ephw_system_bytes(const ephw_system* s, int64_t* bytes) {
  if (!s || !bytes) {
    set_error("ephw_system_bytes: NULL argument");
    return EPHW_EINVAL;
  }
  *bytes = s->bytes;
  return EPHW_OK;
}

ephw_status ephw_set_q_batch(ephw_system* s, int32_t q_batch) {
  if (!s || q_batch < 0 || q_batch > 65535) {
    set_error("ephw_set_q_batch: need a system and 0 <= q_batch <= 65535");
    return EPHW_EINVAL;
  }
  s->q_batch = q_batch;
  return EPHW_OK;
}

ephw_status ephw_profile_enable(ephw_system* s, int32_t enable) {
  if (!s) {
    set_error("ephw_profile_enable: system is NULL");
    return EPHW_EINVAL;
  }
  s->prof.on = enable != 0;
  return EPHW_OK;
}

ephw_status ephw_profile_read(ephw_system* s, double* ms, int64_t* launches) {
  if (!s) {
    set_error("ephw_profile_read: system is NULL");
    return EPHW_EINVAL;
  }
  if (ms)
    for (int i = 0; i < EPHW_NSTAGES; ++i) ms[i] = 0.0;
  if (launches)
    for (int i = 0; i < EPHW_NSTAGES; ++i) launches[i] = 0;
  ephw_status result = EPHW_OK;
  for (auto& r : s->prof.recs) {
    float t = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
      set_error("ephw_profile_read: event query failed");
      result = EPHW_EDEVICE;
    }
    if (r.stage >= 0 && r.stage < EPHW_NSTAGES) {
      if (ms) ms[r.stage] += (double)t;
      if (launches) launches[r.stage] += 1;
    }
    s->prof.pool.push_back(r.a);
    s->prof.pool.push_back(r.b);
  }
  s->prof.recs.clear();
  return result;
}

ephw_status ephw_set_k_tile(ephw_system* s, int32_t k_tile) {
  if (!s || k_tile < 0) {
    set_error("ephw_set_k_tile: need a system and k_tile >= 0");
    return EPHW_EINVAL;
  }
  s->k_tile = k_tile;
  return EPHW_OK;
}

ephw_status ephw_bands(ephw_system* s, const double* k, int64_t nk, double* eps, void* vecs,
                       void* stream) {
  if (!s || (!k && nk > 0) || nk < 0) {
    set_error("ephw_bands: invalid argument");
    return EPHW_EINVAL;
  }
  if (nk == 0) return EPHW_OK;
  hipStream_t st = as_stream(stream);
  const int64_t nw2 = (int64_t)s->nw * s->nw;
  EPHW_TRY(ws_need(s, WS_PH, (size_t)nk * s->nh * 16));
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    EPHW_TRY(phase_matrix(0, k, nk, s->r_h, s->w_h, s->nh, wsp(s, WS_PH), st));
  }
  double* e_out = eps;
  double* v_out = static_cast<double*>(vecs);
  if (!e_out) {
    EPHW_TRY(ws_need(s, WS_EPS, (size_t)nk * s->nw * 8));
    e_out = static_cast<double*>(wsp(s, WS_EPS));
  }
  if (!v_out) {
    EPHW_TRY(ws_need(s, WS_V64, (size_t)nk * nw2 * 16));
    v_out = static_cast<double*>(wsp(s, WS_V64));
  }
  return interp_eigh(s, static_cast<const double*>(wsp(s, WS_PH)), nk, s->nh, s->h_r, s->nw, e_out,
                     v_out, st);
}

ephw_status ephw_phonons(ephw_system* s, const double* q, int64_t nq, double* lam, double* omega,
                         void* evecs, void* stream) {
  if (!s || (!q && nq > 0) || nq < 0) {
    set_error("ephw_phonons: invalid argument");
    return EPHW_EINVAL;
  }
  if (nq == 0) return EPHW_OK;
  hipStream_t st = as_stream(stream);
  const int nm = s->nm;
  EPHW_TRY(ws_need(s, WS_PQC, (size_t)nq * s->nc * 16));
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    EPHW_TRY(phase_matrix(0, q, nq, s->r_c, s->w_c, s->nc, wsp(s, WS_PQC), st));
  }
  double* l_out = lam;
  if (!l_out) {
    EPHW_TRY(ws_need(s, WS_LAM, (size_t)nq * nm * 8));
    l_out = static_cast<double*>(wsp(s, WS_LAM));
  }
  double* e_out = static_cast<double*>(evecs);
  if (!e_out) {
    EPHW_TRY(ws_need(s, WS_E, (size_t)nq * nm * nm * 16));
    e_out = static_cast<double*>(wsp(s, WS_E));
  }
  EPHW_TRY(interp_eigh(s, static_cast<const double*>(wsp(s, WS_PQC)), nq, s->nc, s->c_scaled, nm,
                       l_out, e_out, st));
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st);
    if (omega) EPHW_TRY(abs_sqrt(l_out, omega, nq * nm, st));
  }
  return EPHW_OK;
}

ephw_status ephw_phase_sum_rp(ephw_system* s, const double* q, int64_t nq, int32_t prec, void* out,
                              void* stream) {
  if (!s || ((!q || !out) && nq > 0) || nq < 0) {
    set_error("ephw_phase_sum_rp: invalid argument");
    return EPHW_EINVAL;
  }
  if (prec != EPHW_FP64 && prec != EPHW_FP32 && prec != EPHW_FP32_COMP) {
    set_error("ephw_phase_sum_rp: unknown precision");
    return EPHW_EINVAL;
  }
  const int kind = prec_kind(prec);
  if (kind != s->g_kind) {
    set_error("ephw_phase_sum_rp: precision does not match the stored g (FP64<->c128, FP32<->c64)");
    return EPHW_EINVAL;
  }
  if (nq == 0) return EPHW_OK;
  hipStream_t st = as_stream(stream);
  EPHW_TRY(ws_need(s, WS_PQ, (size_t)nq * s->np * csize(kind)));
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    EPHW_TRY(phase_matrix(kind, q, nq, s->r_p, s->w_p, s->np, wsp(s, WS_PQ), st));
  }
  GemmParams p;
  p.M = nq;
  p.N = s->ne * s->nm * s->nw * s->nw;
  p.K = s->np;
  p.A = wsp(s, WS_PQ);
  p.compensated = prec == EPHW_FP32_COMP;
  p.lda = s->np;
  p.B = s->g;
  p.ldb = p.N;
  p.C = out;
  p.ldc = p.N;
  {
    Stage sg_(s, EPHW_STAGE_RP_GEMM, st);
    return cgemm(kind, p, st);
  }
}

ephw_status ephw_kset_free(ephw_kset* ks) {
  if (!ks) return EPHW_OK;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {ks->k, ks->pk, ks->pkh, ks->eps, ks->v64, ks->vt, ks->dv64, ks->dpk,
                  ks->dv != ks->dv64 ? ks->dv : nullptr};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  dev_release(ks->mem.get(), ks->bytes);
  delete ks;
  return EPHW_OK;
}

ephw_status ephw_kset_create(ephw_system* s, const double* k, int64_t nk, int32_t prec, void* stream,
                             ephw_kset** out) {
  if (!s || !k || !out || nk < 1) {
    set_error("ephw_kset_create: invalid argument (need a system, a k list and nk >= 1)");
    return EPHW_EINVAL;
  }
  if (prec != EPHW_FP64 && prec != EPHW_FP32 && prec != EPHW_FP32_COMP) {
    set_error("ephw_kset_create: unknown precision");
    return EPHW_EINVAL;
  }
  const int kind = prec_kind(prec);
  if (kind != s->g_kind) {
    set_error("ephw_kset_create: precision does not match the stored g (FP64<->c128, FP32<->c64)");
    return EPHW_EINVAL;
  }
  *out = nullptr;
  hipStream_t st = as_stream(stream);
  ephw_kset* ks = new ephw_kset();
  ks->sys = s;
  ks->mem = s->mem;
  ks->nk = nk;
  ks->prec = prec;
  const int64_t nw2 = (int64_t)s->nw * s->nw;
  ephw_status e = EPHW_OK;
  auto alloc = [&](void** p, size_t bytes) {
    ephw_status r = dev_alloc(p, bytes, ks->mem.get());
    if (r == EPHW_OK) ks->bytes += (int64_t)bytes;
    return r;
  };
  auto fail = [&](ephw_status r) {
    ephw_kset_free(ks);
    return r;
  };
  if ((e = alloc((void**)&ks->k, (size_t)nk * 24)) != EPHW_OK) return fail(e);
  if (hipMemcpyAsync(ks->k, k, (size_t)nk * 24, hipMemcpyDeviceToDevice, st) != hipSuccess) {
    set_error("ephw_kset_create: copy of k failed");
    return fail(EPHW_EDEVICE);
  }
  if ((e = alloc(&ks->pk, (size_t)nk * s->ne * csize(kind))) != EPHW_OK) return fail(e);
  if ((e = alloc((void**)&ks->pkh, (size_t)nk * s->nh * 16)) != EPHW_OK) return fail(e);
  if ((e = alloc((void**)&ks->eps, (size_t)nk * s->nw * 8)) != EPHW_OK) return fail(e);
  if ((e = alloc((void**)&ks->v64, (size_t)nk * nw2 * 16)) != EPHW_OK) return fail(e);
  if ((e = alloc(&ks->vt, (size_t)nk * nw2 * csize(kind))) != EPHW_OK) return fail(e);
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    if ((e = phase_matrix(kind, ks->k, nk, s->r_e, s->w_e, s->ne, ks->pk, st)) != EPHW_OK)
      return fail(e);
  }
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st);
    if ((e = phase_matrix(0, ks->k, nk, s->r_h, s->w_h, s->nh, ks->pkh, st)) != EPHW_OK)
      return fail(e);
  }
  if ((e = interp_eigh(s, ks->pkh, nk, s->nh, s->h_r, s->nw, ks->eps, ks->v64, st)) != EPHW_OK)
    return fail(e);
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st);
    if ((e = cast_complex(kind, ks->v64, ks->vt, nk * nw2, st)) != EPHW_OK) return fail(e);
  }
  *out = ks;
  return EPHW_OK;
}

ephw_status ephw_kset_bands(ephw_kset* ks, double* eps, void* vecs, void* stream) {
  if (!ks) {
    set_error("ephw_kset_bands: kset is NULL");
    return EPHW_EINVAL;
  }
  hipStream_t st = as_stream(stream);
  const ephw_system* s = ks->sys;
  if (eps)
    EPHW_HIP(hipMemcpyAsync(eps, ks->eps, (size_t)ks->nk * s->nw * 8, hipMemcpyDeviceToDevice, st));
  if (vecs)
    EPHW_HIP(hipMemcpyAsync(vecs, ks->v64, (size_t)ks->nk * s->nw * s->nw * 16,
                            hipMemcpyDeviceToDevice, st));
  return EPHW_OK;
}

}  // extern "C"

// Static scratch of ephw_interpolate_noalloc: one copy per device, held from
// the library's first use of a device to the end of the process.  Host code
// never passes `scratch` itself to a kernel: it names the host-side shadow,
// not the device copy; scratch_address() looks the device address up.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device buffers of one interpolation call with Nw <= 32, carved from one
// block (the system's workspace, or the static scratch of the entry point
// that allocates nothing) in 256-byte aligned pieces.
struct InterpWs {
  void *pq = nullptr, *u = nullptr, *g = nullptr, *gnu = nullptr, *w = nullptr, *vkq = nullptr;
  double *lam = nullptr, *e = nullptr, *pqc = nullptr, *hk = nullptr, *jwork = nullptr, *pqh = nullptr;
  double *bq = nullptr, *hkq = nullptr, *ekq = nullptr, *vkq64 = nullptr, *loss = nullptr;
  void* gchunk = nullptr;                          // rotated g of a batch for the linewidth (unfused)
  double *om = nullptr, *lwp = nullptr;            // omega [nq][nm]; fused linewidth partials
  size_t bytes = 0;
};

// What a call needs, from its arguments (validated by the caller)
struct InterpReq {
  int64_t nk = 0, nq = 0;
  int32_t prec = 0, qb = 1;
  uint32_t flags = 0;
  bool need_g = false, need_kq_eig = false;
  bool fused = false;        // band rotations in the Re-sum GEMM's epilogue (no W buffer)
  bool lw = false;           // linewidth reduction of the rotated g (no g output)
  LwParams lwp;              // its kernel parameters, from the arguments below
  double temperature = 0, mu = 0, sigma = 0, omega_min = 0;
  int64_t nq_total = 0;
  double* gamma = nullptr;
};

// Whether every q batch of the call can take the fused band epilogue: FP32
// without split phases, rotated output, and a Re-sum GEMM that runs on the
// default 128x128 tile for both the full and the last batch.
bool interp_fusable(const ephw_system* s, const InterpReq& r) {
  if (r.prec != EPHW_FP32 || (r.flags & EPHW_OUT_WANNIER) || !r.need_g) return false;
  const int64_t E = (int64_t)s->nm * s->nw * s->nw, tail = r.nq % r.qb;
  return cgemm_band_fusable(1, r.nk, r.qb * E, s->nw, s->ne, r.qb * E) &&
         (tail == 0 || cgemm_band_fusable(1, r.nk, tail * E, s->nw, s->ne, tail * E));
}

InterpWs interp_layout(const ephw_system* s, const InterpReq& r, char* base) {
  InterpWs w;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  auto takd = [&](size_t bytes) { return reinterpret_cast<double*>(take(bytes)); };
  const int kind = prec_kind(r.prec);
  const size_t cs = csize(kind);
  const int64_t nw = s->nw, nm = s->nm, nw2 = nw * nw, E = nm * nw2, nk = r.nk, nq = r.nq, qb = r.qb;
  w.pq = take((size_t)nq * s->np * cs);
  w.lam = takd((size_t)nq * nm * 8);
  w.e = takd((size_t)nq * nm * nm * 16);
  w.pqc = takd((size_t)nq * s->nc * 16);
  w.hk = takd((size_t)nq * nm * nm * 16);
  const int64_t jw_d = jacobi_work_doubles((int)nm, nq);
  const int64_t jw_kq = r.need_kq_eig ? jacobi_work_doubles((int)nw, qb * nk) : 0;
  const int64_t jw = jw_d > jw_kq ? jw_d : jw_kq;
  if (jw > 0) w.jwork = takd((size_t)jw * 8);
  w.u = take((size_t)nq * nm * nm * cs);
  if (r.need_g) {
    w.g = take((size_t)qb * s->ne * E * cs);
    w.gnu = take((size_t)qb * s->ne * E * cs);
    if (!r.fused) w.w = take((size_t)nk * qb * E * cs);
  }
  if (r.need_kq_eig) {
    w.pqh = takd((size_t)nq * s->nh * 16);
    w.bq = takd((size_t)qb * s->nh * nw2 * 16);
    w.hkq = takd((size_t)qb * nk * nw2 * 16);
    w.vkq64 = takd((size_t)qb * nk * nw2 * 16);
    w.vkq = take((size_t)qb * nk * nw2 * cs);
  }
  if (r.need_kq_eig || r.lw) w.ekq = takd((size_t)qb * nk * nw * 8);
  if (r.flags & EPHW_OUT_LOSS) {
    // per pair (band-rotation kernel) or per tile (fused epilogue)
    const int64_t tiles = ceil_div(nk, 128) * ceil_div(qb * E, 128);
    w.loss = takd((size_t)(tiles > qb * nk ? tiles : qb * nk) * 8);
  }
  if (r.lw) {
    w.om = takd((size_t)nq * nm * 8);
    if (r.fused)
      w.lwp = takd((size_t)cgemm_band_lw_groups(nw, (int)nm, qb * E) * nk * nw * 8 + column_sum_scratch(nk * nw));
    else
      w.gchunk = take((size_t)qb * nk * E * cs);
  }
  w.bytes = off;
  return w;
}

// Host-side checks shared by both interpolation entry points; fills the request.
ephw_status interp_validate(const char* who, ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                            int64_t q_offset, int32_t prec, uint32_t flags, void* g_out, double* band_sum,
                            double* loss, double* eps_kq, double* omega, InterpReq* r) {
  const std::string w(who);
  if (!ks || (!q && nq > 0) || nq < 0 || q_offset < 0) {
    set_error(w + ": invalid argument");
    return EPHW_EINVAL;
  }
  if (prec != ks->prec) {
    set_error(w + ": precision differs from the k-set's");
    return EPHW_EINVAL;
  }
  const uint32_t known = EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS | EPHW_OUT_WANNIER;
  if (flags & ~known) {
    set_error(w + ": unknown output flag");
    return EPHW_EINVAL;
  }
  if (((flags & EPHW_OUT_G) && !g_out) || ((flags & EPHW_OUT_BAND_SUM) && !band_sum) ||
      ((flags & EPHW_OUT_LOSS) && !loss)) {
    set_error(w + ": a requested output buffer is NULL");
    return EPHW_EINVAL;
  }
  if (!(flags & (EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS)) && !eps_kq && !omega) {
    set_error(w + ": nothing requested");
    return EPHW_EINVAL;
  }
  if ((flags & EPHW_OUT_WANNIER) && (flags & EPHW_OUT_LOSS)) {
    set_error(w + ": the loss is defined on the rotated g only");
    return EPHW_EINVAL;
  }
  const bool wannier = (flags & EPHW_OUT_WANNIER) != 0;
  r->nk = ks->nk;
  r->nq = nq;
  r->prec = prec;
  r->flags = flags;
  r->need_g = (flags & (EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS)) != 0;
  r->need_kq_eig = !kq_index && (!wannier || eps_kq);
  return EPHW_OK;
}

// Eq. (7) for Nw <= 32 with every buffer in `w` (see interp_layout).
ephw_status interpolate_small(ephw_kset* ks, const double* q, const int32_t* kq_index, int64_t q_offset,
                              const InterpReq& r, void* g_out, double* band_sum, double* loss, uint64_t loss_seed,
                              double* eps_kq, double* omega, const InterpWs& w, bool stages, hipStream_t st) {
  ephw_system* s = ks->sys;
  const int kind = prec_kind(r.prec);
  const bool comp = r.prec == EPHW_FP32_COMP;
  const uint32_t flags = r.flags;
  const bool wannier = (flags & EPHW_OUT_WANNIER) != 0;
  const int nw = s->nw, nm = s->nm;
  const int64_t nw2 = (int64_t)nw * nw, E = nm * nw2, nk = ks->nk, nq = r.nq;
  const size_t cs = csize(kind);
  const int32_t qb = r.qb;

  // --- per-call q side: Rp phases, D(q) eigensolve, mode vectors ----------
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st, stages);
    EPHW_TRY(phase_matrix(kind, q, nq, s->r_p, s->w_p, s->np, w.pq, st));
  }
  {
    Stage sg_(s, EPHW_STAGE_PHASE, st, stages);
    EPHW_TRY(phase_matrix(0, q, nq, s->r_c, s->w_c, s->nc, w.pqc, st));
  }
  EPHW_TRY(interp_eigh_ws(s, w.pqc, nq, s->nc, s->c_scaled, nm, w.lam, w.e, w.hk, w.jwork, stages, st));
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st, stages);
    if (omega) EPHW_TRY(abs_sqrt(w.lam, omega, nq * nm, st));
    if (r.lw) EPHW_TRY(abs_sqrt(w.lam, w.om, nq * nm, st));
  }
  {
    Stage sg_(s, EPHW_STAGE_OTHER, st, stages);
    EPHW_TRY(mode_vectors(kind, w.e, nq, nm, s->ism, w.u, st));
  }
  if (r.need_kq_eig) {
    Stage sg_(s, EPHW_STAGE_PHASE, st, stages);
    EPHW_TRY(phase_matrix(0, q, nq, s->r_h, nullptr, s->nh, w.pqh, st));
  }

  for (int64_t q0 = 0; q0 < nq; q0 += qb) {
    const int32_t nb = (int32_t)((nq - q0) < qb ? (nq - q0) : qb);
    const double* ekq_b = nullptr;   // bands at k+q of this batch, [nb][nk][nw]
    // bands at k+q: H(k+q) = sum_R e^{2 pi i k.R} (e^{2 pi i q.R} H(R)), then FP64 Jacobi
    if (r.need_kq_eig) {
      Stage sg_(s, EPHW_STAGE_KQ_EIG, st, stages);
      EPHW_TRY(scale_rows_by_phase(w.pqh + 2 * q0 * s->nh, nb, s->h_r, s->nh, nw2, w.bq, st));
      GemmParams h;
      h.M = nk;
      h.N = nw2;
      h.K = s->nh;
      h.batch = nb;
      h.A = ks->pkh;
      h.lda = s->nh;
      h.strideA = 0;
      h.B = w.bq;
      h.ldb = nw2;
      h.strideB = s->nh * nw2;
      h.C = w.hkq;
      h.ldc = nw2;
      h.strideC = nk * nw2;
      EPHW_TRY(cgemm(0, h, st));
      double* ekq = eps_kq ? eps_kq + q0 * nk * nw : w.ekq;
      // FP32 outputs stop the k+q sweeps at an off-diagonal norm of 1e-10 of the
      // total (eigenvalues then exact to ~1e-20 relative, eigenvectors to ~1e-10,
      // far below the complex64 rounding they are cast to); FP64 at 1e-14
      EPHW_TRY(jacobi_eigh(w.hkq, (int64_t)nb * nk, nw, ekq, w.vkq64, w.jwork, s->ctx->status, st,
                           kind == 0 ? 1e-28 : 1e-20));
      EPHW_TRY(cast_complex(kind, w.vkq64, w.vkq, (int64_t)nb * nk * nw2, st));
      ekq_b = ekq;
    } else if ((eps_kq || r.lw) && kq_index) {
      // k+q on the k grid: its bands are the k-set's bands at the indexed point
      Stage sg_(s, EPHW_STAGE_OTHER, st, stages);
      double* ekq = eps_kq ? eps_kq + q0 * nk * nw : w.ekq;
      EPHW_TRY(gather_rows(ks->eps, nk, kq_index + q0 * nk, (int64_t)nb * nk, nw, ekq, s->ctx->status, st));
      ekq_b = ekq;
    }
    if (!r.need_g) continue;
    // Eq. (9): G[q][Re, ka, m', n'] = sum_Rp e^{i q.Rp} g(Re, Rp)
    GemmParams rp;
    rp.M = nb;
    rp.N = s->ne * E;
    rp.K = s->np;
    rp.A = static_cast<const char*>(w.pq) + (size_t)q0 * s->np * cs;
    rp.compensated = comp;
    rp.lda = s->np;
    rp.B = s->g;
    rp.ldb = rp.N;
    rp.C = w.g;
    rp.ldc = rp.N;
    {
      Stage sg_(s, EPHW_STAGE_RP_GEMM, st, stages);
      EPHW_TRY(cgemm(kind, rp, st));
    }
    // mode vectors u(q), hoisted to the g(Re,q) level; output [Re][q][nu][m'][n']
    {
      Stage sg_(s, EPHW_STAGE_MODE_ROT, st, stages);
      EPHW_TRY(mode_rotate(kind, w.g, wannier ? nullptr : static_cast<const char*>(w.u) + (size_t)q0 * nm * nm * cs,
                           w.gnu, s->ne, nb, nm, nw2, st));
    }
    // Eq. (10), Re part: W[k][q nu m' n'] = sum_Re e^{i k.Re} G_nu(Re, q)
    GemmParams re;
    re.M = nk;
    re.N = (int64_t)nb * E;
    re.K = s->ne;
    re.A = ks->pk;
    re.compensated = comp;
    re.lda = s->ne;
    re.B = w.gnu;
    re.ldb = re.N;
    re.C = w.w;
    re.ldc = re.N;
    if (r.fused) {
      // band rotations and epilogues in the GEMM's epilogue: W never leaves the tile
      BandEpilogue& b = re.band;
      b.on = true;
      b.nw = nw;
      b.nm = nm;
      b.nk = nk;
      b.q_global0 = q_offset + q0;
      b.Vk = ks->vt;
      b.Vkq = kq_index ? nullptr : w.vkq;
      b.kq_index = kq_index ? kq_index + q0 * nk : nullptr;
      b.flags = flags & (EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS);
      b.g_out = (flags & EPHW_OUT_G) ? static_cast<char*>(g_out) + (size_t)q0 * nk * E * cs : nullptr;
      b.band_sum = (flags & EPHW_OUT_BAND_SUM) ? band_sum + q0 * nk * nm : nullptr;
      b.loss_partial = w.loss;
      b.loss_seed = loss_seed;
      if (r.lw) {
        b.lw_partial = w.lwp;
        b.eps_k = ks->eps;
        b.eps_kq = ekq_b;
        b.omega = w.om + q0 * nm;
        b.lw = r.lwp;
      }
      b.status = s->ctx->status;
      {
        Stage sg_(s, EPHW_STAGE_RE_GEMM, st, stages);
        EPHW_TRY(cgemm(kind, re, st));
      }
      Stage sg_(s, EPHW_STAGE_OTHER, st, stages);
      if (flags & EPHW_OUT_LOSS) EPHW_TRY(sum_into(w.loss, ceil_div(re.M, 128) * ceil_div(re.N, 128), loss, st));
      if (r.lw) {
        const int64_t groups = cgemm_band_lw_groups(nw, nm, re.N);
        EPHW_TRY(add_column_sums(w.lwp, groups, nk * nw, r.lwp.scale, r.gamma,
                                 w.lwp + cgemm_band_lw_groups(nw, nm, (int64_t)qb * E) * nk * nw, st));
      }
      continue;
    }
    {
      Stage sg_(s, EPHW_STAGE_RE_GEMM, st, stages);
      EPHW_TRY(cgemm(kind, re, st));
    }
    // band rotations V(k+q)^dagger W V(k) and the epilogues
    BandRotateArgs br;
    br.W = w.w;
    br.Vk = wannier ? nullptr : ks->vt;
    br.Vkq = kq_index ? nullptr : w.vkq;
    br.kq_index = kq_index ? kq_index + q0 * nk : nullptr;
    br.nk = nk;
    br.k0 = 0;
    br.nk_tile = nk;
    br.qb = nb;
    br.nm = nm;
    br.nw = nw;
    br.flags = r.lw ? (flags | EPHW_OUT_G) : flags;
    br.g_out = r.lw ? w.gchunk
                    : (flags & EPHW_OUT_G) ? static_cast<char*>(g_out) + (size_t)q0 * nk * E * cs : nullptr;
    br.band_sum = (flags & EPHW_OUT_BAND_SUM) ? band_sum + q0 * nk * nm : nullptr;
    br.loss_partial = w.loss;
    br.loss_seed = loss_seed;
    br.q_global0 = q_offset + q0;
    br.status = s->ctx->status;
    {
      Stage sg_(s, EPHW_STAGE_BAND_ROT, st, stages);
      EPHW_TRY(band_rotate(kind, br, st));
    }
    {
      Stage sg_(s, EPHW_STAGE_OTHER, st, stages);
      if (flags & EPHW_OUT_LOSS) EPHW_TRY(sum_into(w.loss, (int64_t)nb * nk, loss, st));
      if (r.lw) {
        EPHW_TRY(linewidth(kind, w.gchunk, nb, nk, nm, nw, ks->eps, ekq_b, w.om + q0 * nm, r.temperature, r.mu,
                           r.sigma, r.omega_min, r.nq_total, r.gamma, st));
      }
    }
  }
  return EPHW_OK;
}

// Device address of `scratch` on the current device, looked up once per device.
ephw_status scratch_address(int device, char** out) {
  static std::mutex mu;
  static std::map<int, char*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return EPHW_OK;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
    return EPHW_EDEVICE;
  }
  addr[device] = static_cast<char*>(p);
  *out = static_cast<char*>(p);
  return EPHW_OK;
}

}  // namespace

extern "C" {

ephw_status ephw_interpolate(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                             int64_t q_offset, int32_t prec, uint32_t flags, void* g_out,
                             double* band_sum, double* loss, uint64_t loss_seed, double* eps_kq,
                             double* omega, void* stream) {
  InterpReq r;
  EPHW_TRY(interp_validate("ephw_interpolate", ks, q, nq, kq_index, q_offset, prec, flags, g_out, band_sum, loss,
                           eps_kq, omega, &r));
  if (nq == 0) return EPHW_OK;
  ephw_system* s = ks->sys;
  if (s->nw > 32)
    return interpolate_large(ks, q, nq, kq_index, q_offset, flags, g_out, band_sum, loss, loss_seed, eps_kq, omega,
                             as_stream(stream));
  r.qb = pick_q_batch(s, ks->nk, nq, prec_kind(prec));
  r.fused = interp_fusable(s, r);
  const size_t need = interp_layout(s, r, nullptr).bytes;
  EPHW_TRY(ws_need(s, WS_ARENA, need));
  const InterpWs w = interp_layout(s, r, static_cast<char*>(wsp(s, WS_ARENA)));
  return interpolate_small(ks, q, kq_index, q_offset, r, g_out, band_sum, loss, loss_seed, eps_kq, omega, w, true,
                           as_stream(stream));
}

ephw_status ephw_interpolate_linewidth(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                       double temperature, double mu, double sigma, double omega_min,
                                       int64_t nq_total, double* gamma, void* stream) {
  if (!ks || (!q && nq > 0) || nq < 0 || !gamma || nq_total < 1 || !(temperature > 0.0) || !(sigma > 0.0) ||
      !(omega_min >= 0.0) || !std::isfinite(mu) || !std::isfinite(temperature) || !std::isfinite(sigma) ||
      !std::isfinite(omega_min)) {
    set_error("ephw_interpolate_linewidth: invalid argument");
    return EPHW_EINVAL;
  }
  if (nq == 0) return EPHW_OK;
  ephw_system* s = ks->sys;
  if (s->nw > 32) {
    set_error("ephw_interpolate_linewidth: systems with more than 32 bands are not supported");
    return EPHW_EUNSUPPORTED;
  }
  InterpReq r;
  r.nk = ks->nk;
  r.nq = nq;
  r.prec = ks->prec;
  r.flags = 0;
  r.need_g = true;
  r.need_kq_eig = !kq_index;
  r.lw = true;
  r.lwp = lw_params(temperature, mu, sigma, omega_min, nq_total);
  r.temperature = temperature;
  r.mu = mu;
  r.sigma = sigma;
  r.omega_min = omega_min;
  r.nq_total = nq_total;
  r.gamma = gamma;
  r.qb = pick_q_batch(s, ks->nk, nq, prec_kind(ks->prec));
  r.fused = interp_fusable(s, r);
  const size_t need = interp_layout(s, r, nullptr).bytes;
  EPHW_TRY(ws_need(s, WS_ARENA, need));
  const InterpWs w = interp_layout(s, r, static_cast<char*>(wsp(s, WS_ARENA)));
  return interpolate_small(ks, q, kq_index, 0, r, nullptr, nullptr, nullptr, 0, nullptr, nullptr, w, true,
                           as_stream(stream));
}

ephw_status ephw_interpolate_noalloc(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                     int64_t q_offset, int32_t prec, uint32_t flags, void* g_out, double* band_sum,
                                     double* loss, uint64_t loss_seed, double* eps_kq, double* omega, void* stream) {
  InterpReq r;
  EPHW_TRY(interp_validate("ephw_interpolate_noalloc", ks, q, nq, kq_index, q_offset, prec, flags, g_out, band_sum,
                           loss, eps_kq, omega, &r));
  if (nq == 0) return EPHW_OK;
  ephw_system* s = ks->sys;
  if (s->nw > 32) {
    set_error("ephw_interpolate_noalloc: systems with more than 32 bands are not supported");
    return EPHW_EUNSUPPORTED;
  }
  // the largest q batch (up to the one ephw_interpolate would take) whose
  // buffers fit the scratch; the per-call buffers grow with nq, not with it
  int32_t qb = pick_q_batch(s, ks->nk, nq, prec_kind(prec));
  for (;;) {
    r.qb = qb;
    r.fused = interp_fusable(s, r);
    if (interp_layout(s, r, nullptr).bytes <= kScratchBytes) break;
    if (qb == 1) {
      set_error("ephw_interpolate_noalloc: the call needs " + std::to_string(interp_layout(s, r, nullptr).bytes) +
                " bytes of scratch at one q per batch, more than the " + std::to_string(kScratchBytes) +
                " bytes the library holds");
      return EPHW_ENOMEM;
    }
    qb = qb / 2 > 0 ? qb / 2 : 1;
  }
  char* base = nullptr;
  EPHW_TRY(scratch_address(s->ctx->device, &base));
  const InterpWs w = interp_layout(s, r, base);
  return interpolate_small(ks, q, kq_index, q_offset, r, g_out, band_sum, loss, loss_seed, eps_kq, omega, w, false,
                           as_stream(stream));
}

ephw_status ephw_degenerate_sums(int32_t prec, const void* g, int64_t nq, int64_t nk, int32_t nm, int32_t nw,
                                 const double* eps_kq, const double* eps_k, const double* lam, double rel_tol,
                                 double* out, void* stream) {
  if (prec != EPHW_FP64 && prec != EPHW_FP32 && prec != EPHW_FP32_COMP) {
    set_error("ephw_degenerate_sums: unknown precision");
    return EPHW_EINVAL;
  }
  if (nq < 0 || nk < 0 || nw < 1 || nw > 256 || nm < 1 || nm > 258 || !(rel_tol >= 0.0) ||
      rel_tol > 1e300) {
    set_error("ephw_degenerate_sums: sizes or tolerance out of range");
    return EPHW_EINVAL;
  }
  if (nq * nk == 0) return EPHW_OK;
  if (!g || !eps_kq || !eps_k || !lam || !out) {
    set_error("ephw_degenerate_sums: a buffer is NULL");
    return EPHW_EINVAL;
  }
  return degenerate_sums(prec == EPHW_FP64 ? 0 : 1, g, nq, nk, nm, nw, eps_kq, eps_k, lam, rel_tol, out,
                         as_stream(stream));
}

ephw_status ephw_linewidth(int32_t prec, const void* g, int64_t nq, int64_t nk, int32_t nm, int32_t nw,
                           const double* eps_k, const double* eps_kq, const double* omega, double temperature,
                           double mu, double sigma, double omega_min, int64_t nq_total, double* gamma,
                           void* stream) {
  if (prec != EPHW_FP64 && prec != EPHW_FP32 && prec != EPHW_FP32_COMP) {
    set_error("ephw_linewidth: unknown precision");
    return EPHW_EINVAL;
  }
  if (nq < 0 || nk < 0 || nw < 1 || nw > 256 || nm < 1 || nm > 258 || nq_total < 1 || !(temperature > 0.0) ||
      !(sigma > 0.0) || !(omega_min >= 0.0) || !std::isfinite(mu) || !std::isfinite(temperature) ||
      !std::isfinite(sigma) || !std::isfinite(omega_min)) {
    set_error("ephw_linewidth: sizes or parameters out of range");
    return EPHW_EINVAL;
  }
  if (nq * nk == 0) return EPHW_OK;
  if (!g || !eps_k || !eps_kq || !omega || !gamma) {
    set_error("ephw_linewidth: a buffer is NULL");
    return EPHW_EINVAL;
  }
  return linewidth(prec == EPHW_FP64 ? 0 : 1, g, nq, nk, nm, nw, eps_k, eps_kq, omega, temperature, mu, sigma,
                   omega_min, nq_total, gamma, as_stream(stream));
}

}  // extern "C"
