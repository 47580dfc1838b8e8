// Internal handle types and helpers shared by the libephw host sources.
#pragma once

#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "gemm.h"
#include "kernels.h"

namespace ephw {

// Device memory a context's systems, k-sets and batches hold, against an
// optional cap (limit 0 = none).  Allocations that would pass the cap fail
// with EPHW_ENOMEM before hipMalloc is called.
struct MemBudget {
  int64_t limit = 0;
  std::atomic<int64_t> used{0};
};

// grow-only device buffer; reallocation waits for the device to go idle
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

inline ephw_status dev_alloc(void** p, size_t bytes, MemBudget* budget = nullptr) {
  if (bytes == 0) bytes = 16;
  *p = nullptr;
  if (budget && budget->limit > 0 && budget->used.load() + (int64_t)bytes > budget->limit) {
    set_error("allocation of " + std::to_string(bytes) + " bytes would exceed the context's device-memory limit of " +
              std::to_string(budget->limit) + " bytes (" + std::to_string(budget->used.load()) + " in use)");
    return EPHW_ENOMEM;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    *p = nullptr;
    return EPHW_ENOMEM;
  }
  if (budget) budget->used += (int64_t)bytes;
  return EPHW_OK;
}

inline void dev_release(MemBudget* budget, int64_t bytes) {
  if (budget) budget->used -= bytes;
}

inline ephw_status grow(DevBuf& b, size_t bytes, int64_t* owner_bytes, MemBudget* budget) {
  if (b.bytes >= bytes && b.p) return EPHW_OK;
  if (b.p) {
    EPHW_HIP(hipDeviceSynchronize());
    EPHW_HIP(hipFree(b.p));
    *owner_bytes -= (int64_t)b.bytes;
    dev_release(budget, (int64_t)b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  EPHW_TRY(dev_alloc(&b.p, bytes, budget));
  b.bytes = bytes;
  *owner_bytes += (int64_t)bytes;
  return EPHW_OK;
}

template <typename X>
inline ephw_status upload(X** dst, const X* src, size_t count, int64_t* owner_bytes, MemBudget* budget) {
  void* p = nullptr;
  EPHW_TRY(dev_alloc(&p, count * sizeof(X), budget));
  *owner_bytes += (int64_t)(count * sizeof(X));
  EPHW_HIP(hipMemcpy(p, src, count * sizeof(X), hipMemcpyHostToDevice));
  *dst = static_cast<X*>(p);
  return EPHW_OK;
}

inline int prec_kind(int32_t prec) { return prec == EPHW_FP64 ? 0 : 1; }
inline size_t csize(int kind) { return kind == 0 ? 16 : 8; }

// FP64 interpolation + eigensolve: out_eps [n][dim], out_v c128 [n][dim][dim]
// from A = phases [n][nr] (c128) and B = R-space matrices [nr][dim*dim] (c128),
// with caller-given buffers: hk [n][dim][dim] c128 and, for dim > 32, jwork of
// jacobi_work_doubles(dim, n) doubles
ephw_status interp_eigh_ws(ephw_system* s, const double* phase, int64_t n, int64_t nr, const double* mats, int dim,
                           double* out_eps, double* out_v, double* hk, double* jwork, bool stages, hipStream_t st);

ephw_status interpolate_large(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index, int64_t q_offset,
                              uint32_t flags, void* g_out, double* band_sum, double* loss, uint64_t loss_seed,
                              double* eps_kq, double* omega, hipStream_t st);

}  // namespace ephw

using namespace ephw;

struct ephw_ctx {
  int device = 0;
  // device words: [0] status bits raised by kernels, [1] sweep limit of the
  // Jacobi eigensolves (read by the kernels at run time)
  uint32_t* status = nullptr;
  // shared with every object made on the context, so that objects freed
  // after the context (in any order) still release their bytes safely
  std::shared_ptr<MemBudget> mem = std::make_shared<MemBudget>();
};

enum WsSlot {
  WS_PQ, WS_PQH, WS_PQC, WS_D, WS_LAM, WS_E, WS_U, WS_G, WS_GNU, WS_W, WS_BQ, WS_HKQ,
  WS_EKQ, WS_VKQ64, WS_VKQ, WS_JWORK, WS_LOSS, WS_PH, WS_HK, WS_EPS, WS_V64,
  // adjoint and large-band rotations
  WS_ADJ_A, WS_ADJ_B, WS_ADJ_C, WS_DPQ, WS_DE64, WS_DU, WS_VKBAR, WS_PAIRS, WS_DKACC, WS_GBAR, WS_GNUBAR, WS_T,
  WS_YBAR, WS_Z, WS_WBAR, WS_PAIRBAR, WS_OFF, WS_UBAR, WS_SPLIT, WS_SPLITB, WS_DOTPART,
  // coarse Bloch -> Wannier transform
  WS_CPK, WS_UINV,
  // energy-window screen and the pair-list interpolation
  WS_WINDOW, WS_PAIRSET,
  // the buffers of an interpolation call (Nw <= 32) in one block
  WS_ARENA, WS_COUNT
};

// HIP-event brackets around the stages of a call, summed on request
struct Profiler {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

struct ephw_system {
  ephw_ctx* ctx = nullptr;
  std::shared_ptr<MemBudget> mem;   // the context's budget
  Profiler prof;
  int nw = 0, na = 0, nm = 0;
  int64_t ne = 0, np = 0, nh = 0, nc = 0;
  int g_kind = 0;  // 0 = c128, 1 = c64
  int32_t *r_e = nullptr, *r_p = nullptr, *r_h = nullptr, *r_c = nullptr;
  double *w_e = nullptr, *w_p = nullptr, *w_h = nullptr, *w_c = nullptr;
  double* h_r = nullptr;      // c128 [nh][nw][nw]
  double* c_scaled = nullptr; // c128 [nc][nm][nm] = C / sqrt(M M')
  double* ism = nullptr;      // [nm] 1/sqrt(M_kappa) per mode index
  void* g = nullptr;
  int32_t q_batch = 0;
  int32_t k_tile = 0;
  int64_t bytes = 0;
  DevBuf ws[WS_COUNT];
  // pinned host staging of per-call descriptors (pair lists), reused once the
  // copy recorded by `staged` has completed
  void* stage_host = nullptr;
  size_t stage_bytes = 0;
  hipEvent_t staged = nullptr;
};

struct ephw_kset {
  ephw_system* sys = nullptr;
  std::shared_ptr<MemBudget> mem;   // the context's budget
  int64_t nk = 0;
  int32_t prec = 0;
  int64_t bytes = 0;
  double* k = nullptr;      // [nk][3]
  void* pk = nullptr;       // T [nk][ne]
  double* pkh = nullptr;    // c128 [nk][nh]
  double* eps = nullptr;    // [nk][nw]
  double* v64 = nullptr;    // c128 [nk][nw][nw]
  void* vt = nullptr;       // T [nk][nw][nw]
  // derivatives for the adjoint, made on first use
  double* dv64 = nullptr;   // c128 [3][nk][nw][nw]: dV/dk_d
  void* dv = nullptr;       // T copy (aliases dv64 for FP64)
  void* dpk = nullptr;      // T [3][nk][ne]: 2 pi i Re_d e^{2 pi i k.Re}
};

// Records a start event on construction and a stop event on destruction
// when the system's profiler is on.
struct Stage {
  Profiler* p;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Stage(ephw_system* s, int stage_, hipStream_t st_, bool enabled = true) : p(&s->prof), stage(stage_), st(st_) {
    if (enabled && p->on) {
      a = p->get();
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~Stage() {
    if (p->on && a) {
      hipEvent_t b = p->get();
      if (b) {
        (void)hipEventRecord(b, st);
        p->recs.push_back({stage, a, b});
      } else {
        p->pool.push_back(a);
      }
    }
  }
};

inline void* wsp(ephw_system* s, WsSlot slot) { return s->ws[slot].p; }

inline ephw_status ws_need(ephw_system* s, WsSlot slot, size_t bytes) {
  return grow(s->ws[slot], bytes, &s->bytes, s->mem.get());
}

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

