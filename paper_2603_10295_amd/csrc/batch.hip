// Many systems in one pass: per-item shapes from the autotuner, rounds of
// grouped launches over all systems, the pass captured into a HIP graph.
//
// Item i runs its units (q batch j, k tile t) in order, one unit per round;
// a unit with t == 0 first needs the Eq. (9) GEMM and the mode rotation of
// q batch j.  Every stage of a round is one launch over all items that take
// part in it: the GEMM stages are persistent grouped GEMMs (one launch per
// tile configuration; a fixed grid of resident workgroups takes the tiles of
// every item from per-XCD work queues, zeroed by a kernel at the start of the
// pass); the other stages are grouped block grids, the band rotations one
// launch per kernel instance and LDS size.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <sstream>

#include "internal.h"

namespace {

struct ItemPlan {
  ephw_batch_item in{};
  ephw_system* sys = nullptr;
  ephw_kset* ks = nullptr;
  int nw = 0, nm = 0;
  int64_t ne = 0, np = 0, nc = 0, nk = 0, nq = 0, E = 0;
  int32_t qb = 0, kt = 0, cfg_rp = 0, cfg_re = 0;
  int64_t nqb = 0, nkt = 0;
  BandPlan band;       // band-rotation work split
  int nwb = 4;         // band-rotation kernel instance
  // workspace
  void* pq = nullptr;      // T [nq][np]
  double* pqc = nullptr;   // c128 [nq][nc]
  double* dq = nullptr;    // c128 [nq][nm][nm]
  double* lam = nullptr;   // [nq][nm]
  double* ev = nullptr;    // c128 [nq][nm][nm]
  void* u = nullptr;       // T [nq][nm][nm]
  void* G = nullptr;       // T [qb][ne*E]
  void* Gnu = nullptr;     // T [ne][qb*E]
  void* W = nullptr;       // T [kt][qb*E]
  double* lossp = nullptr; // [qb*kt]
  // runs its units in rounds of its own, after the grouped rounds, with the
  // sweep buffers (G, Gnu, W, lossp) in a region shared by all such items
  bool solo = false;
  size_t q_bytes() const;      // per-q buffers, computed once per pass
  size_t sweep_bytes() const;  // buffers of one unit
  size_t bytes() const { return q_bytes() + sweep_bytes(); }
  int64_t units() const { return nqb * nkt; }
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Launch {
  enum Kind { PHASE, GEMM, PGEMM, EIGH, MODEVEC, MODE, BAND, SUM } kind;
  GemmParams gp;               // PGEMM: one plain GEMM (a solo item's phase sum)
  int prec = 0;
  int cfg = 0;                 // GEMM: tile configuration of every problem in the launch
  int grid = 0;                // GEMM: persistent workgroups
  int qidx = -1;               // GEMM: index of its kGroupQueues work-queue counters
  const void* jobs = nullptr;  // device descriptor array
  int n = 0;
  int64_t count = 0;           // total tiles (GEMM) or blocks
  size_t lds = 0;
  int order = 0;               // EIGH: largest matrix order among the jobs
  // PHASE / MODEVEC: direct arguments
  int item = -1;
};

}  // namespace

struct ephw_batch {
  ephw_ctx* ctx = nullptr;
  std::shared_ptr<MemBudget> mem;   // the context's budget
  int kind = 0;
  std::vector<ItemPlan> items;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* desc = nullptr;
  size_t desc_bytes = 0;
  std::vector<Launch> launches;
  int* queues = nullptr;       // kGroupQueues counters per GEMM launch (in the descriptor buffer)
  int nqueue = 0;              // GEMM launches
  int rounds = 0;
  int cus = 256;
  bool use_graph = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

size_t ItemPlan::q_bytes() const {
  const size_t cs = csize(sys->g_kind);
  size_t b = 0;
  b += align256((size_t)nq * np * cs);
  b += align256((size_t)nq * nc * 16);
  b += align256((size_t)nq * nm * nm * 16);
  b += align256((size_t)nq * nm * 8);
  b += align256((size_t)nq * nm * nm * 16);
  b += align256((size_t)nq * nm * nm * cs);
  return b;
}

size_t ItemPlan::sweep_bytes() const {
  const size_t cs = csize(sys->g_kind);
  size_t b = 0;
  b += align256((size_t)qb * ne * E * cs);
  b += align256((size_t)qb * ne * E * cs);
  b += align256((size_t)kt * qb * E * cs);
  b += align256((size_t)qb * kt * 8);
  return b;
}

// per-q buffers at qbase (q_bytes), sweep buffers at sbase (sweep_bytes)
void carve(ItemPlan& it, char* qbase, char* sbase) {
  const size_t cs = csize(it.sys->g_kind);
  char* base = qbase;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align256(b);
    return p;
  };
  it.pq = take((size_t)it.nq * it.np * cs);
  it.pqc = reinterpret_cast<double*>(take((size_t)it.nq * it.nc * 16));
  it.dq = reinterpret_cast<double*>(take((size_t)it.nq * it.nm * it.nm * 16));
  it.lam = reinterpret_cast<double*>(take((size_t)it.nq * it.nm * 8));
  it.ev = reinterpret_cast<double*>(take((size_t)it.nq * it.nm * it.nm * 16));
  it.u = take((size_t)it.nq * it.nm * it.nm * cs);
  base = sbase;
  off = 0;
  it.G = take((size_t)it.qb * it.ne * it.E * cs);
  it.Gnu = take((size_t)it.qb * it.ne * it.E * cs);
  it.W = take((size_t)it.kt * it.qb * it.E * cs);
  it.lossp = reinterpret_cast<double*>(take((size_t)it.qb * it.kt * 8));
}

// k points per tile that keep the item's sweep buffers within `cap` bytes
int32_t k_tile_for(const ItemPlan& it, int32_t qb, int64_t cap) {
  const double cs = (double)csize(it.sys->g_kind);
  const double fixed = 2.0 * qb * it.ne * it.E * cs;
  const double per_k = (double)qb * it.E * cs + 8.0 * qb;
  if (fixed >= (double)cap) return 0;
  int64_t kt = (int64_t)(((double)cap - fixed) / per_k);
  if (kt >= it.nk) return (int32_t)it.nk;
  if (kt >= 128) kt -= kt % 64;  // whole 64-row tiles
  return (int32_t)kt;
}

void set_shape(ItemPlan& it, int32_t qb, int32_t kt) {
  it.qb = qb;
  it.kt = kt;
  it.cfg_rp = qb >= 128 ? 0 : 1;
  it.cfg_re = kt >= 128 ? 0 : 1;
  it.nqb = ceil_div(it.nq, qb);
  it.nkt = ceil_div(it.nk, kt);
}

std::string shape_key(int kind, const ItemPlan& it) {
  char buf[256];
  snprintf(buf, sizeof(buf), "gfx950|%s|nw%d|nm%d|ne%lld|np%lld|nk%lld|nq%lld", kind == 0 ? "fp64" : "fp32",
           it.nw, it.nm, (long long)it.ne, (long long)it.np, (long long)it.nk, (long long)it.nq);
  return buf;
}

// tuned shapes: one JSON object per line {"key": "...", "qb": n, "kt": n}
std::map<std::string, std::pair<int, int>> read_cache(const char* path) {
  std::map<std::string, std::pair<int, int>> m;
  if (!path) return m;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t k0 = line.find("\"key\": \"");
    const size_t q0 = line.find("\"qb\": ");
    const size_t t0 = line.find("\"kt\": ");
    if (k0 == std::string::npos || q0 == std::string::npos || t0 == std::string::npos) continue;
    const size_t k1 = line.find('"', k0 + 8);
    if (k1 == std::string::npos) continue;
    m[line.substr(k0 + 8, k1 - k0 - 8)] = {atoi(line.c_str() + q0 + 6), atoi(line.c_str() + t0 + 6)};
  }
  return m;
}

void append_cache(const char* path, const std::string& key, int qb, int kt, double us_per_pair) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << "{\"key\": \"" << key << "\", \"qb\": " << qb << ", \"kt\": " << kt << ", \"us_per_kpair\": " << us_per_pair
    << "}\n";
}

// ---- one unit of one item, launched directly (autotuning) ------------------
ephw_status unit_direct(ItemPlan& it, int kind, int64_t j, int64_t t, hipStream_t st, uint32_t* status) {
  const int64_t q0 = j * it.qb, nb = std::min<int64_t>(it.qb, it.nq - q0);
  const int64_t k0 = t * it.kt, kl = std::min<int64_t>(it.kt, it.nk - k0);
  const size_t cs = csize(kind);
  GemmParams rp;
  rp.M = nb;
  rp.N = it.ne * it.E;
  rp.K = it.np;
  rp.A = static_cast<const char*>(it.pq) + (size_t)q0 * it.np * cs;
  rp.lda = it.np;
  rp.B = it.sys->g;
  rp.ldb = rp.N;
  rp.C = it.G;
  rp.ldc = rp.N;
  EPHW_TRY(cgemm(kind, rp, st));
  EPHW_TRY(mode_rotate(kind, it.G, static_cast<const char*>(it.u) + (size_t)q0 * it.nm * it.nm * cs, it.Gnu,
                       it.ne, (int)nb, it.nm, (int64_t)it.nw * it.nw, st));
  GemmParams re;
  re.M = kl;
  re.N = nb * it.E;
  re.K = it.ne;
  re.A = static_cast<const char*>(it.ks->pk) + (size_t)k0 * it.ne * cs;
  re.lda = it.ne;
  re.B = it.Gnu;
  re.ldb = re.N;
  re.C = it.W;
  re.ldc = re.N;
  EPHW_TRY(cgemm(kind, re, st));
  BandRotateArgs br;
  br.W = it.W;
  br.Vk = it.ks->vt;
  br.Vkq = nullptr;
  br.kq_index = it.in.kq_index + q0 * it.nk;
  br.nk = it.nk;
  br.k0 = k0;
  br.nk_tile = kl;
  br.qb = (int)nb;
  br.nm = it.nm;
  br.nw = it.nw;
  br.flags = EPHW_OUT_LOSS;
  br.g_out = nullptr;
  br.band_sum = nullptr;
  br.loss_partial = it.lossp;
  br.loss_seed = 0;
  br.q_global0 = q0;
  br.status = status;
  return band_rotate(kind, br, st);
}

ephw_status tune_item(ItemPlan& it, int kind, int64_t cap, bool measure, hipStream_t st, uint32_t* status,
                      double* us_per_kpair) {
  std::vector<int32_t> cands;
  for (int32_t qb : {128, 64, 32, 16}) {
    const int32_t q = (int32_t)std::min<int64_t>(qb, it.nq);
    if (std::find(cands.begin(), cands.end(), q) == cands.end() && k_tile_for(it, q, cap) >= std::min<int64_t>(16, it.nk))
      cands.push_back(q);
  }
  // items whose two g(Re,q) sweeps at 16 q do not fit the cap take fewer q
  for (int32_t qb = 8; cands.empty() && qb >= 1; qb /= 2) {
    const int32_t q = (int32_t)std::min<int64_t>(qb, it.nq);
    if (k_tile_for(it, q, cap) >= std::min<int64_t>(16, it.nk)) cands.push_back(q);
  }
  if (cands.empty()) {
    set_error("ephw_batch_create: an item does not fit the per-item workspace cap");
    return EPHW_ENOMEM;
  }
  *us_per_kpair = 0.0;
  if (!measure) {
    set_shape(it, cands[0], k_tile_for(it, cands[0], cap));
    return EPHW_OK;
  }
  // the largest candidate's buffers serve every candidate
  int32_t best_q = cands[0];
  double best = 1e300;
  size_t need = 0;
  for (int32_t q : cands) {
    set_shape(it, q, k_tile_for(it, q, cap));
    need = std::max(need, it.bytes());
  }
  void* tmp = nullptr;
  EPHW_TRY(dev_alloc(&tmp, need, it.sys->mem.get()));
  hipEvent_t a = nullptr, b = nullptr;
  ephw_status rc = EPHW_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = EPHW_EDEVICE;
  for (size_t ci = 0; ci < cands.size() && rc == EPHW_OK; ++ci) {
    const int32_t q = cands[ci];
    set_shape(it, q, k_tile_for(it, q, cap));
    carve(it, static_cast<char*>(tmp), static_cast<char*>(tmp) + it.q_bytes());
    // phases and mode vectors of the first q batch (values only matter for timing)
    rc = phase_matrix(kind, it.in.q, std::min<int64_t>(q, it.nq), it.sys->r_p, it.sys->w_p, it.np, it.pq, st);
    if (rc == EPHW_OK) rc = hipMemsetAsync(it.u, 0, (size_t)q * it.nm * it.nm * csize(kind), st) == hipSuccess
                                ? EPHW_OK : EPHW_EDEVICE;
    for (int rep = 0; rep < 2 && rc == EPHW_OK; ++rep) {
      (void)hipEventRecord(a, st);
      rc = unit_direct(it, kind, 0, 0, st, status);
      (void)hipEventRecord(b, st);
    }
    if (rc != EPHW_OK) break;
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      rc = EPHW_EDEVICE;
      break;
    }
    const double pairs = (double)std::min<int64_t>(q, it.nq) * std::min<int64_t>(it.kt, it.nk);
    const double us = 1e3 * ms / pairs * 1e3;  // microseconds per 1000 pairs
    if (us < best) {
      best = us;
      best_q = q;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(st);
  (void)hipFree(tmp);
  dev_release(it.sys->mem.get(), (int64_t)need);
  if (rc != EPHW_OK) return rc;
  set_shape(it, best_q, k_tile_for(it, best_q, cap));
  *us_per_kpair = best;
  return EPHW_OK;
}

// ---- descriptor staging ----------------------------------------------------
struct HostDesc {
  std::vector<char> bytes;
  struct Fix {
    size_t off;
    Launch* l;
  };
  template <typename J>
  size_t add(const std::vector<J>& v) {
    const size_t off = align256(bytes.size());
    bytes.resize(off + v.size() * sizeof(J));
    memcpy(bytes.data() + off, v.data(), v.size() * sizeof(J));
    return off;
  }
};

ephw_status issue(ephw_batch* bt, hipStream_t st) {
  uint32_t* status = bt->ctx->status;
  // the grouped GEMMs' work queues start from zero on every pass
  EPHW_TRY(cgemm_grouped_reset(bt->queues, bt->nqueue * kGroupQueues, st));
  for (const Launch& l : bt->launches) {
    switch (l.kind) {
      case Launch::PHASE: {
        ItemPlan& it = bt->items[l.item];
        EPHW_TRY(phase_matrix(bt->kind, it.in.q, it.nq, it.sys->r_p, it.sys->w_p, it.np, it.pq, st));
        EPHW_TRY(phase_matrix(0, it.in.q, it.nq, it.sys->r_c, it.sys->w_c, it.nc, it.pqc, st));
        break;
      }
      case Launch::MODEVEC: {
        ItemPlan& it = bt->items[l.item];
        EPHW_TRY(mode_vectors(bt->kind, it.ev, it.nq, it.nm, it.sys->ism, it.u, st));
        break;
      }
      case Launch::GEMM:
        EPHW_TRY(cgemm_grouped(l.prec, l.cfg, static_cast<const GroupProblem*>(l.jobs), l.n, l.count,
                               (int)std::min<int64_t>(l.grid, l.count), bt->queues + l.qidx * kGroupQueues, st));
        break;
      case Launch::PGEMM:
        EPHW_TRY(cgemm(l.prec, l.gp, st));
        break;
      case Launch::EIGH:
        EPHW_TRY(jacobi_eigh_grouped(static_cast<const EighJob*>(l.jobs), l.n, l.count, l.order, status, st));
        break;
      case Launch::MODE:
        EPHW_TRY(mode_rotate_grouped(bt->kind, static_cast<const ModeRotateJob*>(l.jobs), l.n, l.count, l.lds, st));
        break;
      case Launch::BAND:
        EPHW_TRY(band_rotate_grouped(bt->kind, l.cfg, static_cast<const BandRotateJob*>(l.jobs), l.n, l.count, l.lds,
                                     st));
        break;
      case Launch::SUM:
        EPHW_TRY(sum_into_grouped(static_cast<const SumJob*>(l.jobs), l.n, st));
        break;
    }
  }
  return EPHW_OK;
}

// Builds the launch list of one pass; descriptor arrays are staged in `hd`
// and their offsets fixed up once the device copy exists.
void build_launches(ephw_batch* bt, HostDesc& hd, std::vector<std::pair<size_t, size_t>>& fix) {
  const int kind = bt->kind;
  const size_t cs = csize(kind);
  auto push = [&](Launch l, size_t off) {
    bt->launches.push_back(l);
    fix.push_back({bt->launches.size() - 1, off});
  };
  // grouped GEMM launches: one per tile configuration present
  auto push_gemm = [&](int prec, const std::vector<GroupProblem>& all) {
    for (int cfg = 0; cfg < 2; ++cfg) {
      std::vector<GroupProblem> probs;
      for (const GroupProblem& p : all)
        if (p.cfg == cfg) probs.push_back(p);
      if (probs.empty()) continue;
      Launch l;
      l.kind = Launch::GEMM;
      l.prec = prec;
      l.cfg = cfg;
      l.grid = bt->cus * cgemm_grouped_blocks_per_cu(prec, cfg);
      l.n = (int)probs.size();
      l.count = cgemm_grouped_layout(prec, probs.data(), l.n);
      l.qidx = bt->nqueue++;
      push(l, hd.add(probs));
    }
  };
  // a solo item's phase sums as plain GEMMs: the tile (or, for at most 16
  // rows, the streaming kernel) chosen for its own shape, as one at a time
  auto push_plain = [&](int prec, const std::vector<GroupProblem>& all) {
    for (const GroupProblem& p : all) {
      Launch l;
      l.kind = Launch::PGEMM;
      l.prec = prec;
      l.gp.M = p.M;
      l.gp.N = p.N;
      l.gp.K = p.K;
      l.gp.A = p.A;
      l.gp.lda = p.lda;
      l.gp.B = p.B;
      l.gp.ldb = p.ldb;
      l.gp.C = p.C;
      l.gp.ldc = p.ldc;
      bt->launches.push_back(l);
    }
  };
  // q side: phases per item, D(q) GEMMs (one grouped launch), eigensolves (one
  // grouped launch), mode vectors per item
  for (size_t i = 0; i < bt->items.size(); ++i) {
    Launch l;
    l.kind = Launch::PHASE;
    l.item = (int)i;
    bt->launches.push_back(l);
  }
  {
    std::vector<GroupProblem> probs;
    for (auto& it : bt->items) {
      GroupProblem p;
      p.M = it.nq;
      p.N = (int64_t)it.nm * it.nm;
      p.K = it.nc;
      p.A = it.pqc;
      p.lda = it.nc;
      p.B = it.sys->c_scaled;
      p.ldb = p.N;
      p.C = it.dq;
      p.ldc = p.N;
      p.cfg = 1;
      probs.push_back(p);
    }
    push_gemm(0, probs);
  }
  {
    std::vector<EighJob> jobs;
    int64_t base = 0;
    int order = 0;
    for (auto& it : bt->items) {
      order = std::max(order, it.nm);
      EighJob j;
      j.H = it.dq;
      j.eps = it.lam;
      j.V = it.ev;
      j.n = it.nm;
      j.count = it.nq;
      j.block_base = base;
      base += it.nq;
      jobs.push_back(j);
    }
    Launch l;
    l.kind = Launch::EIGH;
    l.n = (int)jobs.size();
    l.count = base;
    l.order = order;
    push(l, hd.add(jobs));
  }
  for (size_t i = 0; i < bt->items.size(); ++i) {
    Launch l;
    l.kind = Launch::MODEVEC;
    l.item = (int)i;
    bt->launches.push_back(l);
  }
  // rounds: the grouped items together, then each solo item on its own
  bt->rounds = 0;
  auto emit_rounds = [&](const std::vector<ItemPlan*>& members) {
    int64_t rounds = 0;
    for (ItemPlan* m : members) rounds = std::max(rounds, m->units());
    const bool plain = members.size() == 1 && members[0]->solo;
    bt->rounds += (int)rounds;
    for (int64_t r = 0; r < rounds; ++r) {
      std::vector<GroupProblem> rp, re;
      std::vector<ModeRotateJob> mj;
      std::vector<BandRotateJob> bj;
      std::vector<int> bj_cls;
      std::vector<size_t> bj_lds;
      std::vector<SumJob> sj;
      int64_t mblocks = 0;
      size_t mlds = 0;
      for (ItemPlan* mp : members) {
        ItemPlan& it = *mp;
        if (r >= it.units()) continue;
        const int64_t j = r / it.nkt, t = r % it.nkt;
        const int64_t q0 = j * it.qb, nb = std::min<int64_t>(it.qb, it.nq - q0);
        const int64_t k0 = t * it.kt, kl = std::min<int64_t>(it.kt, it.nk - k0);
        const int64_t nw2 = (int64_t)it.nw * it.nw;
        if (t == 0) {
          GroupProblem p;
          p.M = nb;
          p.N = it.ne * it.E;
          p.K = it.np;
          p.A = static_cast<const char*>(it.pq) + (size_t)q0 * it.np * cs;
          p.lda = it.np;
          p.B = it.sys->g;
          p.ldb = p.N;
          p.C = it.G;
          p.ldc = p.N;
          p.cfg = it.cfg_rp;
          rp.push_back(p);
          ModeRotateJob m;
          m.G = it.G;
          m.u = static_cast<const char*>(it.u) + (size_t)q0 * it.nm * it.nm * cs;
          m.Gnu = it.Gnu;
          m.ne = it.ne;
          m.nw2 = nw2;
          m.qb = (int)nb;
          m.nm = it.nm;
          m.block_base = mblocks;
          mblocks += nb * ceil_div(it.ne * nw2, 256);
          mlds = std::max(mlds, (size_t)it.nm * it.nm * cs);
          mj.push_back(m);
        }
        GroupProblem p;
        p.M = kl;
        p.N = nb * it.E;
        p.K = it.ne;
        p.A = static_cast<const char*>(it.ks->pk) + (size_t)k0 * it.ne * cs;
        p.lda = it.ne;
        p.B = it.Gnu;
        p.ldb = p.N;
        p.C = it.W;
        p.ldc = p.N;
        p.cfg = it.cfg_re;
        re.push_back(p);
        BandRotateJob b;
        BandRotateArgs& br = b.args;
        br.W = it.W;
        br.Vk = it.ks->vt;
        br.Vkq = nullptr;
        br.kq_index = it.in.kq_index + q0 * it.nk;
        br.nk = it.nk;
        br.k0 = k0;
        br.nk_tile = kl;
        br.qb = (int)nb;
        br.nm = it.nm;
        br.nw = it.nw;
        br.flags = it.in.flags;
        br.g_out = (it.in.flags & EPHW_OUT_G) ? static_cast<char*>(it.in.g_out) + (size_t)q0 * it.nk * it.E * cs
                                              : nullptr;
        br.band_sum = (it.in.flags & EPHW_OUT_BAND_SUM) ? it.in.band_sum + q0 * it.nk * it.nm : nullptr;
        br.loss_partial = (it.in.flags & EPHW_OUT_LOSS) ? it.lossp : nullptr;
        br.loss_seed = it.in.loss_seed;
        br.q_global0 = q0;
        br.status = bt->ctx->status;
        b.P = it.band.P;
        b.nuc = it.band.nuc;
        b.block_base = 0;
        bj.push_back(b);
        bj_cls.push_back(it.nwb);
        bj_lds.push_back(it.band.lds);
        if (it.in.flags & EPHW_OUT_LOSS) sj.push_back(SumJob{it.lossp, nb * kl, it.in.loss});
      }
      if (!rp.empty()) {
        if (plain)
          push_plain(kind, rp);
        else
          push_gemm(kind, rp);
        Launch m;
        m.kind = Launch::MODE;
        m.n = (int)mj.size();
        m.count = mblocks;
        m.lds = mlds;
        push(m, hd.add(mj));
      }
      {
        if (plain)
          push_plain(kind, re);
        else
          push_gemm(kind, re);
        // one band-rotation launch per kernel instance (band count rounded up
        // to a multiple of 4) and LDS size (in 8 KB steps): a launch runs at the
        // occupancy its largest LDS request allows
        std::vector<std::pair<int, size_t>> keys;
        for (size_t i = 0; i < bj.size(); ++i) {
          const std::pair<int, size_t> key{bj_cls[i], ceil_div((int64_t)bj_lds[i], 8192)};
          if (std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
        }
        std::sort(keys.begin(), keys.end());
        for (const auto& key : keys) {
          const int cls = key.first;
          std::vector<BandRotateJob> part;
          int64_t blocks = 0;
          size_t lds = 0;
          for (size_t i = 0; i < bj.size(); ++i) {
            if (bj_cls[i] != cls || (size_t)ceil_div((int64_t)bj_lds[i], 8192) != key.second) continue;
            BandRotateJob jb = bj[i];
            const int64_t nblk = (int64_t)jb.args.qb * ceil_div(jb.args.nk_tile, (int64_t)jb.P);
            jb.block_base = blocks;
            blocks += nblk;
            lds = std::max(lds, bj_lds[i]);
            part.push_back(jb);
          }
          if (part.empty()) continue;
          Launch b;
          b.kind = Launch::BAND;
          b.cfg = cls;
          b.n = (int)part.size();
          b.count = blocks;
          b.lds = lds;
          push(b, hd.add(part));
        }
      }
      if (!sj.empty()) {
        Launch l;
        l.kind = Launch::SUM;
        l.n = (int)sj.size();
        l.count = (int64_t)sj.size();
        push(l, hd.add(sj));
      }
    }
  };
  std::vector<ItemPlan*> grouped;
  for (auto& it : bt->items)
    if (!it.solo) grouped.push_back(&it);
  emit_rounds(grouped);
  for (auto& it : bt->items)
    if (it.solo) emit_rounds({&it});
}

}  // namespace

extern "C" {

ephw_status ephw_batch_free(ephw_batch* b) {
  if (!b) return EPHW_OK;
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->ws) {
    (void)hipFree(b->ws);
    dev_release(b->mem.get(), (int64_t)b->ws_bytes);
  }
  if (b->desc) {
    (void)hipFree(b->desc);
    dev_release(b->mem.get(), (int64_t)b->desc_bytes);
  }
  delete b;
  return EPHW_OK;
}

ephw_status ephw_batch_create(ephw_ctx* ctx, const ephw_batch_item* items, int32_t n,
                              const ephw_batch_options* opt, void* stream, ephw_batch** out) {
  if (!ctx || !items || n < 1 || !out) {
    set_error("ephw_batch_create: need a context, n >= 1 items and an output handle");
    return EPHW_EINVAL;
  }
  *out = nullptr;
  ephw_batch_options o{};
  o.use_graph = 1;
  if (opt) o = *opt;
  hipStream_t st = as_stream(stream);
  ephw_batch* bt = new ephw_batch();
  bt->ctx = ctx;
  bt->mem = ctx->mem;
  auto fail = [&](ephw_status e) {
    ephw_batch_free(bt);
    return e;
  };
  for (int32_t i = 0; i < n; ++i) {
    const ephw_batch_item& in = items[i];
    if (!in.ks || (!in.q && in.nq > 0) || in.nq < 0 || !in.kq_index) {
      set_error("ephw_batch_create: item " + std::to_string(i) + " needs a k-set, a q list and a k+q index");
      return fail(EPHW_EINVAL);
    }
    const uint32_t known = EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS;
    if ((in.flags & ~known) || !(in.flags & known) || ((in.flags & EPHW_OUT_G) && !in.g_out) ||
        ((in.flags & EPHW_OUT_BAND_SUM) && !in.band_sum) || ((in.flags & EPHW_OUT_LOSS) && !in.loss)) {
      set_error("ephw_batch_create: item " + std::to_string(i) + " has inconsistent output flags/buffers");
      return fail(EPHW_EINVAL);
    }
    ItemPlan it;
    it.in = in;
    it.ks = in.ks;
    it.sys = in.ks->sys;
    const int kind = prec_kind(in.ks->prec);
    if (i == 0) bt->kind = kind;
    if (kind != bt->kind || in.ks->prec == EPHW_FP32_COMP) {
      set_error("ephw_batch_create: all items must share one precision (FP64 or FP32)");
      return fail(EPHW_EINVAL);
    }
    if (it.sys->ctx != ctx) {
      set_error("ephw_batch_create: item system belongs to another context");
      return fail(EPHW_EINVAL);
    }
    it.nw = it.sys->nw;
    it.nm = it.sys->nm;
    if (it.nw > 32 || it.nm > 24) {
      set_error("ephw_batch_create: batched items need nw <= 32 and nm <= 24");
      return fail(EPHW_EUNSUPPORTED);
    }
    it.ne = it.sys->ne;
    it.np = it.sys->np;
    it.nc = it.sys->nc;
    it.nk = in.ks->nk;
    it.nq = in.nq;
    it.E = (int64_t)it.nm * it.nw * it.nw;
    if (!cgemm_grouped_fits(kind, it.np, it.ne * it.E) || !cgemm_grouped_fits(kind, it.ne, 128 * it.E) ||
        !cgemm_grouped_fits(0, it.nc, (int64_t)it.nm * it.nm)) {
      set_error("ephw_batch_create: item " + std::to_string(i) + " is too large for the grouped GEMM");
      return fail(EPHW_EUNSUPPORTED);
    }
    it.band = band_rotate_plan(kind, it.nw, it.nm);
    it.nwb = band_rotate_class(it.nw);
    bt->items.push_back(it);
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) == hipSuccess && cus > 0)
    bt->cus = cus;
  // Sweep-buffer cap per item: the given per-item cap, else what the item's
  // largest unit (128 q, every k) needs, at most 8 GiB.  If the items
  // together want more than half of the free HBM, the largest items run solo
  // (their rounds after the grouped ones, one item at a time, in one shared
  // sweep region) until the rest fit beside that region; only if even the
  // smallest items do not fit are the grouped items' caps scaled down (not
  // below 1 GiB).
  std::vector<int64_t> caps(bt->items.size(), o.item_workspace_bytes);
  if (o.item_workspace_bytes <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      set_error("ephw_batch_create: hipMemGetInfo failed");
      return fail(EPHW_EDEVICE);
    }
    const double gib = (double)(1 << 30);
    const double budget = o.workspace_budget_bytes > 0 ? (double)o.workspace_budget_bytes : 0.5 * (double)fr;
    for (size_t i = 0; i < bt->items.size(); ++i) {
      const ItemPlan& it = bt->items[i];
      const double cs = (double)csize(bt->kind), qb = (double)std::min<int64_t>(128, std::max<int64_t>(1, it.nq));
      const double full = 2.0 * qb * it.ne * it.E * cs + (double)it.nk * qb * (it.E * cs + 8.0) + 64.0 * (1 << 20);
      caps[i] = (int64_t)std::max(gib, std::min(8.0 * gib, full));
    }
    std::vector<size_t> order(bt->items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return caps[a] > caps[b]; });
    double want = 0.0, solo_region = 0.0;
    for (int64_t c : caps) want += (double)c;
    for (size_t r = 0; r < order.size() && want + solo_region > budget; ++r) {
      ItemPlan& it = bt->items[order[r]];
      if (it.nq == 0) continue;
      it.solo = true;
      want -= (double)caps[order[r]];
      solo_region = std::max(solo_region, (double)caps[order[r]]);
    }
    const double room = budget - solo_region;
    if (want > room)
      for (size_t i = 0; i < caps.size(); ++i)
        if (!bt->items[i].solo) caps[i] = (int64_t)std::max(gib, (double)caps[i] * std::max(room, 0.0) / want);
    // never below what one q with a 16-point k tile needs
    for (size_t i = 0; i < bt->items.size(); ++i) {
      const ItemPlan& it = bt->items[i];
      const double cs = (double)csize(bt->kind);
      const double least = 2.0 * it.ne * it.E * cs + (double)std::min<int64_t>(16, it.nk) * (it.E * cs + 8.0) +
                           (double)(1 << 20);
      caps[i] = std::max(caps[i], (int64_t)least);
    }
  }
  // shapes: cache, else tune (or heuristics)
  auto cache = read_cache(o.tune_cache);
  for (size_t i = 0; i < bt->items.size(); ++i) {
    ItemPlan& it = bt->items[i];
    const int64_t cap = caps[i];
    if (it.nq == 0) {  // nothing to do: smallest buffers, no units
      set_shape(it, 1, 1);
      continue;
    }
    const std::string key = shape_key(bt->kind, it);
    auto f = cache.find(key);
    if (f != cache.end() && f->second.first > 0 && f->second.second > 0 &&
        k_tile_for(it, f->second.first, cap) >= f->second.second) {
      set_shape(it, f->second.first, f->second.second);
      continue;
    }
    double us = 0.0;
    ephw_status e = tune_item(it, bt->kind, cap, o.tune != 0, st, ctx->status, &us);
    if (e != EPHW_OK) return fail(e);
    if (o.tune) {
      append_cache(o.tune_cache, key, it.qb, it.kt, us);
      cache[key] = {it.qb, it.kt};
    }
  }
  // workspace: every item's per-q buffers and the grouped items' sweep
  // buffers side by side, then one sweep region that the solo items share
  // (their rounds run one item after another in stream order)
  size_t total = 0, solo_bytes = 0;
  for (auto& it : bt->items) {
    total += it.q_bytes();
    if (it.solo)
      solo_bytes = std::max(solo_bytes, it.sweep_bytes());
    else
      total += it.sweep_bytes();
  }
  ephw_status e = dev_alloc(&bt->ws, total + solo_bytes, bt->mem.get());
  if (e != EPHW_OK) return fail(e);
  bt->ws_bytes = total + solo_bytes;
  {
    char* base = static_cast<char*>(bt->ws);
    char* shared = base + total;
    size_t off = 0;
    for (auto& it : bt->items) {
      char* q = base + off;
      off += it.q_bytes();
      if (it.solo) {
        carve(it, q, shared);
      } else {
        carve(it, q, base + off);
        off += it.sweep_bytes();
      }
    }
  }
  // launch list + descriptors
  HostDesc hd;
  std::vector<std::pair<size_t, size_t>> fix;
  build_launches(bt, hd, fix);
  const size_t qoff = align256(hd.bytes.size());
  hd.bytes.resize(qoff + (size_t)std::max(1, bt->nqueue) * kGroupQueues * sizeof(int), 0);
  if ((e = dev_alloc(&bt->desc, hd.bytes.size(), bt->mem.get())) != EPHW_OK) return fail(e);
  bt->desc_bytes = hd.bytes.size();
  bt->queues = reinterpret_cast<int*>(static_cast<char*>(bt->desc) + qoff);
  if (hipMemcpy(bt->desc, hd.bytes.data(), hd.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("ephw_batch_create: descriptor upload failed");
    return fail(EPHW_EDEVICE);
  }
  for (auto& fx : fix) bt->launches[fx.first].jobs = static_cast<char*>(bt->desc) + fx.second;
  // large-LDS band rotations need the attribute before any capture
  for (int cls = 4; cls <= 32; cls += 4) {
    size_t blds = 0;
    for (auto& l : bt->launches)
      if (l.kind == Launch::BAND && l.cfg == cls) blds = std::max(blds, l.lds);
    if ((e = band_rotate_grouped_prepare(bt->kind, cls, blds)) != EPHW_OK) return fail(e);
  }
  bt->use_graph = o.use_graph != 0;
  if (bt->use_graph) {
    if (hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking) != hipSuccess) {
      set_error("ephw_batch_create: capture stream");
      return fail(EPHW_EDEVICE);
    }
    if (hipStreamBeginCapture(bt->cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
      set_error("ephw_batch_create: hipStreamBeginCapture failed");
      return fail(EPHW_EDEVICE);
    }
    ephw_status ie = issue(bt, bt->cap);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(bt->cap, &g);
    if (ie != EPHW_OK) {
      if (g) (void)hipGraphDestroy(g);
      return fail(ie);
    }
    if (ce != hipSuccess || !g) {
      set_error(std::string("ephw_batch_create: capture failed: ") + hipGetErrorString(ce));
      return fail(EPHW_EDEVICE);
    }
    bt->graph = g;
    if (hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0) != hipSuccess) {
      set_error("ephw_batch_create: hipGraphInstantiate failed");
      return fail(EPHW_EDEVICE);
    }
  }
  *out = bt;
  return EPHW_OK;
}

ephw_status ephw_batch_run(ephw_batch* b, void* stream) {
  if (!b) {
    set_error("ephw_batch_run: batch is NULL");
    return EPHW_EINVAL;
  }
  hipStream_t st = as_stream(stream);
  if (b->exec) {
    EPHW_HIP(hipGraphLaunch(b->exec, st));
    return EPHW_OK;
  }
  return issue(b, st);
}

ephw_status ephw_batch_shape(const ephw_batch* b, int32_t i, int32_t* q_batch, int32_t* k_tile, int32_t* cfg_rp,
                             int32_t* cfg_re) {
  if (!b || i < 0 || i >= (int32_t)b->items.size()) {
    set_error("ephw_batch_shape: no such item");
    return EPHW_EINVAL;
  }
  const ItemPlan& it = b->items[i];
  if (q_batch) *q_batch = it.qb;
  if (k_tile) *k_tile = it.kt;
  if (cfg_rp) *cfg_rp = it.cfg_rp;
  if (cfg_re) *cfg_re = it.cfg_re;
  return EPHW_OK;
}

ephw_status ephw_batch_solo(const ephw_batch* b, int32_t i, int32_t* solo) {
  if (!b || !solo || i < 0 || i >= (int32_t)b->items.size()) {
    set_error("ephw_batch_solo: no such item or NULL output");
    return EPHW_EINVAL;
  }
  *solo = b->items[i].solo ? 1 : 0;
  return EPHW_OK;
}

ephw_status ephw_batch_stats(const ephw_batch* b, int32_t* rounds, int32_t* launches) {
  if (!b) {
    set_error("ephw_batch_stats: batch is NULL");
    return EPHW_EINVAL;
  }
  int32_t nl = 0;
  for (auto& l : b->launches) nl += (l.kind == Launch::PHASE) ? 2 : 1;
  if (rounds) *rounds = b->rounds;
  if (launches) *launches = nl;
  return EPHW_OK;
}

}  // extern "C"
