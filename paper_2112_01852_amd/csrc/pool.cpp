// Serving pool: continuous batching of domain-wall CG solves.
//
// Requests (each with its own lattice, Ls, mass, gauge field and source) wait
// in FIFO order until their device memory fits the caller's arena and a slot
// is free; then they are admitted: their links and source are packed into
// arena memory and they join the pool's group (group.h). Every step waits
// for the previous round, retires the requests that finished in it (their
// solution unpacked into the caller's buffer, their arena memory returned),
// admits what now fits, and launches one round for all members at once on
// the caller's stream: one launch per step of the CG iteration for every
// request, replayed from a graph captured when the pool was created. After
// creation the pool allocates no device memory: everything lives in the
// arena, sub-allocated here (first fit, 256-byte aligned). Site tables are
// shared by the requests of one lattice shape and kept until the arena needs
// the room.
//
// A request's arithmetic depends only on its own data (its own reductions,
// its own sequence of iterations and reliable updates), so its result is the
// same whether it runs alone or among others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "common.h"
#include "group.h"
#include "solver.h"

namespace qdwf {

std::vector<double> build_local_matrices(const qdwf_action& a);

namespace {

// First-fit sub-allocator of the arena (offsets; 256-byte granules).
struct Arena {
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
  void init(size_t bytes) {
    size = bytes & ~(size_t)255;
    used = 0;
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = al256(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = al256(bytes ? bytes : 1);
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct GeoKey {
  int L[4], bc[4];
  bool operator<(const GeoKey& o) const {
    return std::lexicographical_compare(L, L + 4, o.L, o.L + 4) ||
           (std::equal(L, L + 4, o.L) && std::lexicographical_compare(bc, bc + 4, o.bc, o.bc + 4));
  }
};

struct GeoEntry {
  std::shared_ptr<const GeomTables> tables;
  size_t off = 0, bytes = 0;
  int users = 0;
};

struct PoolRequest {
  uint64_t id;
  qdwf_action act;
  qdwf_solve_params prm;
  const void* U;
  const void* b;
  void* x_out;
  // while admitted
  qdwf_ctx* ctx = nullptr;   // host object; its arrays live in the arena
  size_t off = 0, bytes = 0;
  int slot = -1;
  GroupMember m = {};
  std::chrono::steady_clock::time_point t_admit;
  // once finished
  int rc = QDWF_OK;
  qdwf_solve_stats stats = {};
};

// Per-request device block: context arrays (the 5D-local matrices, FP64 links
// and the inner precision's links), the solver workspace, x_o and b_o.
struct ReqLayout {
  CtxLayout ctx;
  size_t ws, xo, bo, total;
};

ReqLayout req_layout(const qdwf_action& a, int inner) {
  ReqLayout R;
  R.ctx = ctx_layout(a, false, (1u << QDWF_F64) | (1u << inner), false);
  const long n = (long)a.L[0] * a.L[1] * a.L[2] * a.L[3] / 2 * a.Ls * 24;
  size_t o = R.ctx.total;
  R.ws = o;
  o += al256(solver_layout(n, 1, inner).total);
  R.xo = o;
  o += al256(8 * (size_t)n);
  R.bo = o;
  o += al256(8 * (size_t)n);
  R.total = o;
  return R;
}

size_t geo_bytes(const qdwf_action& a) { return ctx_layout(a, true, 0u, false).geom_bytes; }

size_t mats_bytes(int Ls) { return al256((size_t)MAT_COUNT * 2 * Ls * Ls * (8 + 4)); }
constexpr int kMatsLsMax = 32;

}  // namespace
}  // namespace qdwf

struct qdwf_pool {
  int device = 0;
  char* arena = nullptr;
  qdwf::Arena alloc;
  size_t peak = 0;
  int max_slots = 0;
  qdwf_solve_params prm = {};
  qdwf::GroupEngine* engine = nullptr;
  size_t table_off = 0, states_off = 0, overhead = 0;
  qdwf::RhsState* d_states = nullptr;
  qdwf::RhsState* h_states = nullptr;   // pinned copy after each round
  char* h_mats = nullptr;                // pinned staging of the matrices, one area per slot
  hipEvent_t ev = nullptr;
  hipStream_t capture = nullptr;
  bool in_flight = false;
  std::vector<char> slot_busy;
  std::map<qdwf::GeoKey, qdwf::GeoEntry> geo;
  std::deque<qdwf::PoolRequest*> queue;
  std::vector<qdwf::PoolRequest*> active;
  std::map<uint64_t, qdwf::PoolRequest*> finished;
  std::map<uint64_t, int> where;   // 0 queued, 1 active, 2 finished
  uint64_t next_id = 1;
};

using namespace qdwf;

namespace {

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&prev) == hipSuccess) (void)hipSetDevice(d);
  }
  ~Dev() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void note_peak(qdwf_pool* p) { p->peak = std::max(p->peak, p->alloc.used); }

// Frees the arena room of site tables no admitted request uses.
void evict_unused_geometry(qdwf_pool* p) {
  for (auto it = p->geo.begin(); it != p->geo.end();) {
    if (it->second.users == 0) {
      p->alloc.release(it->second.off, it->second.bytes);
      it = p->geo.erase(it);
    } else {
      ++it;
    }
  }
}

// Site tables of this request's shape in the arena (built and uploaded the
// first time the shape is admitted). Returns QDWF_EBUSY when they do not fit.
int acquire_geometry(qdwf_pool* p, const qdwf_action& a, hipStream_t st, GeoEntry** out) {
  GeoKey k;
  std::copy(a.L, a.L + 4, k.L);
  std::copy(a.bc, a.bc + 4, k.bc);
  auto it = p->geo.find(k);
  if (it != p->geo.end()) {
    *out = &it->second;
    return QDWF_OK;
  }
  GeoEntry e;
  e.bytes = geo_bytes(a);
  if (!p->alloc.alloc(e.bytes, &e.off)) {
    evict_unused_geometry(p);
    if (!p->alloc.alloc(e.bytes, &e.off)) return QDWF_EBUSY;
  }
  note_peak(p);
  try {
    // every Ls of a lattice shape shares its tables: the traversal is the
    // environment's or the default, never a per-Ls tuned one
    e.tables = build_geometry(a.L, a.bc, pick_traversal(a.L, 0, p->device));
  } catch (const std::bad_alloc&) {
    p->alloc.release(e.off, e.bytes);
    return fail(QDWF_ENOMEM, "host allocation of the site tables failed");
  }
  // upload once per lattice shape, ordered on the pool's stream after the
  // work that may still read this arena room (a retired request's unpack);
  // the host tables stay alive in the cache
  const CtxLayout L = ctx_layout(a, true, 0u, false);
  char* base = p->arena + e.off;
  const GeomTables& G = *e.tables;
  hipError_t err =
      hipMemcpyAsync(base + L.nbr, G.nbr.data(), 4 * G.nbr.size(), hipMemcpyHostToDevice, st);
  if (err == hipSuccess)
    err = hipMemcpyAsync(base + L.site_lex, G.site_lex.data(), 4 * G.site_lex.size(),
                         hipMemcpyHostToDevice, st);
  if (err == hipSuccess)
    err = hipMemcpyAsync(base + L.idx, G.idx.data(), 4 * G.idx.size(), hipMemcpyHostToDevice, st);
  if (err != hipSuccess) {
    p->alloc.release(e.off, e.bytes);
    return fail(QDWF_EDEVICE, "upload of the site tables failed: %s", hipGetErrorString(err));
  }
  *out = &(p->geo[k] = e);
  return QDWF_OK;
}

void release(qdwf_pool* p, PoolRequest* r) {
  if (r->ctx) {
    GeoKey k;
    std::copy(r->act.L, r->act.L + 4, k.L);
    std::copy(r->act.bc, r->act.bc + 4, k.bc);
    auto it = p->geo.find(k);
    if (it != p->geo.end()) it->second.users -= 1;
    delete r->ctx;
    r->ctx = nullptr;
  }
  if (r->bytes) p->alloc.release(r->off, r->bytes);
  r->bytes = 0;
  if (r->slot >= 0) p->slot_busy[r->slot] = 0;
  r->slot = -1;
}

// Admits r if it fits: QDWF_OK (admitted), QDWF_EBUSY (does not fit now),
// or an error (the request fails).
int admit(qdwf_pool* p, PoolRequest* r, hipStream_t st) {
  int slot = -1;
  for (int i = 0; i < p->max_slots; ++i)
    if (!p->slot_busy[i]) { slot = i; break; }
  if (slot < 0) return QDWF_EBUSY;
  const ReqLayout R = req_layout(r->act, p->prm.inner_prec);
  size_t off = 0;
  if (!p->alloc.alloc(R.total, &off)) {
    evict_unused_geometry(p);
    if (!p->alloc.alloc(R.total, &off)) return QDWF_EBUSY;
  }
  GeoEntry* ge = nullptr;
  int rc = acquire_geometry(p, r->act, st, &ge);
  if (rc) {
    p->alloc.release(off, R.total);
    return rc;
  }
  note_peak(p);
  r->off = off;
  r->bytes = R.total;
  r->slot = slot;
  p->slot_busy[slot] = 1;
  qdwf_ctx* c = new (std::nothrow) qdwf_ctx();
  if (!c) return fail(QDWF_ENOMEM, "host allocation failed");
  r->ctx = c;
  ge->users += 1;
  c->act = r->act;
  c->device = p->device;
  Geom& g = c->g;
  for (int mu = 0; mu < 4; ++mu) g.L[mu] = r->act.L[mu];
  g.Ls = r->act.Ls;
  g.V = g.L[0] * g.L[1] * g.L[2] * g.L[3];
  g.Vh = g.V / 2;
  g.n5h = (long)g.Vh * g.Ls;
  c->geo = ge->tables;
  for (int k = 0; k < 4; ++k) c->tile[k] = c->geo->tile[k];
  for (int k = 0; k < 2; ++k) c->order[k] = c->geo->order[k];
  const CtxLayout GL = ctx_layout(r->act, true, 0u, false);
  char* gbase = p->arena + ge->off;
  c->d_nbr = reinterpret_cast<int32_t*>(gbase + GL.nbr);
  c->d_site_lex = reinterpret_cast<int32_t*>(gbase + GL.site_lex);
  c->d_idx = reinterpret_cast<int32_t*>(gbase + GL.idx);
  char* base = p->arena + off;
  place_arrays(c, base, R.ctx);
  // 5D-local matrices through the slot's pinned staging (asynchronous)
  try {
    c->h_mat = build_local_matrices(r->act);
  } catch (const std::bad_alloc&) {
    return fail(QDWF_ENOMEM, "host allocation failed");
  }
  char* hm = p->h_mats + (size_t)slot * mats_bytes(kMatsLsMax);
  const size_t nm = c->h_mat.size();
  std::memcpy(hm, c->h_mat.data(), 8 * nm);
  float* hm32 = reinterpret_cast<float*>(hm + 8 * nm);
  for (size_t i = 0; i < nm; ++i) hm32[i] = (float)c->h_mat[i];
  QDWF_HIP(hipMemcpyAsync(c->d_mat64, hm, 8 * nm, hipMemcpyHostToDevice, st));
  QDWF_HIP(hipMemcpyAsync(c->d_mat32, hm32, 4 * nm, hipMemcpyHostToDevice, st));
  if ((rc = launch_pack_links(c, r->U, QDWF_F64, st))) return rc;
  c->gauge_set = true;
  double* xo = reinterpret_cast<double*>(base + R.xo);
  double* bo = reinterpret_cast<double*>(base + R.bo);
  if ((rc = launch_pack(c, bo, QDWF_F64, p->prm.layout, r->b, QDWF_F64, QDWF_ODD, 1, st, false)))
    return rc;
  GroupMember& m = r->m;
  m.ctx = c;
  m.xo = xo;
  m.bo = bo;
  m.ws = base + R.ws;
  m.st = p->d_states + slot;
  m.tol = r->prm.tol;
  m.delta = r->prm.delta;
  m.max_iter = r->prm.max_iter;
  if ((rc = p->engine->start_member(m, st))) return rc;
  r->t_admit = std::chrono::steady_clock::now();
  return QDWF_OK;
}

void finish(qdwf_pool* p, PoolRequest* r, int rc) {
  r->rc = rc;
  p->finished[r->id] = r;
  p->where[r->id] = 2;
}

int status_code(int s) {
  switch (s) {
    case ST_DONE: return QDWF_OK;
    case ST_NOTCONV: return QDWF_ENOTCONV;
    default: return QDWF_ENAN;
  }
}

bool validate_params(const qdwf_solve_params& p) {
  return p.tol > 0.0 && p.tol < 1.0 && p.delta >= 0.0 && p.delta < 1.0;
}

size_t overhead_bytes(int max_slots) {
  return group_table_bytes() + al256(sizeof(RhsState) * (size_t)max_slots);
}

size_t request_total(const qdwf_action& a, int inner) {
  return req_layout(a, inner).total + al256(geo_bytes(a));
}

}  // namespace

extern "C" {

size_t qdwf_request_bytes(const qdwf_action* act, const qdwf_solve_params* params) {
  if (!act || !params || params->inner_prec < QDWF_F64 || params->inner_prec > QDWF_BF16) return 0;
  return request_total(*act, params->inner_prec);
}

size_t qdwf_pool_overhead_bytes(int max_slots) {
  if (max_slots < 1 || max_slots > kGroupMax) return 0;
  return overhead_bytes(max_slots);
}

int qdwf_pool_create(int device, void* arena, size_t arena_bytes, int max_slots,
                     const qdwf_solve_params* params, qdwf_pool** out) {
  if (!out || !params) return fail(QDWF_EINVAL, "null argument");
  *out = nullptr;
  if (!arena) return fail(QDWF_EINVAL, "arena is NULL");
  if (reinterpret_cast<uintptr_t>(arena) & 255) return fail(QDWF_EINVAL, "arena must be 256-byte aligned");
  if (max_slots < 1 || max_slots > kGroupMax)
    return fail(QDWF_EINVAL, "max_slots %d out of [1, %d]", max_slots, kGroupMax);
  const qdwf_solve_params& pr = *params;
  if (pr.inner_prec < QDWF_F64 || pr.inner_prec > QDWF_BF16) return fail(QDWF_EINVAL, "inner precision");
  if (pr.layout != QDWF_RIRI && pr.layout != QDWF_RRII) return fail(QDWF_EINVAL, "layout");
  const int k = pr.check_every > 0 ? pr.check_every : 8;
  if (k > 64) return fail(QDWF_EINVAL, "check_every %d out of [1, 64]", k);
  if (arena_bytes < overhead_bytes(max_slots))
    return fail(QDWF_EINVAL, "arena of %zu bytes is smaller than the pool's own %zu", arena_bytes,
                overhead_bytes(max_slots));
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(QDWF_EINVAL, "device %d not available", device);
  Dev dg(device);
  qdwf_pool* p = new (std::nothrow) qdwf_pool();
  if (!p) return fail(QDWF_ENOMEM, "host allocation failed");
  p->device = device;
  p->arena = reinterpret_cast<char*>(arena);
  p->alloc.init(arena_bytes);
  p->max_slots = max_slots;
  p->prm = pr;
  p->prm.check_every = k;
  p->slot_busy.assign(max_slots, 0);
  int rc = QDWF_OK;
  auto bail = [&](int code) {
    qdwf_pool_destroy(p);
    return code;
  };
  (void)p->alloc.alloc(group_table_bytes(), &p->table_off);
  (void)p->alloc.alloc(sizeof(RhsState) * (size_t)max_slots, &p->states_off);
  p->overhead = p->alloc.used;
  note_peak(p);
  p->d_states = reinterpret_cast<RhsState*>(p->arena + p->states_off);
  if (hipHostMalloc(reinterpret_cast<void**>(&p->h_states), sizeof(RhsState) * max_slots) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&p->h_mats), mats_bytes(kMatsLsMax) * max_slots) != hipSuccess) {
    return bail(fail(QDWF_ENOMEM, "pinned host allocation failed"));
  }
  if (hipEventCreateWithFlags(&p->ev, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(QDWF_EDEVICE, "event or stream creation failed"));
  if ((rc = GroupEngine::create(device, pr.inner_prec, pr.layout, k, p->arena + p->table_off,
                                p->capture, &p->engine)))
    return bail(rc);
  *out = p;
  return QDWF_OK;
}

int qdwf_pool_destroy(qdwf_pool* pool) {
  if (!pool) return QDWF_OK;
  Dev dg(pool->device);
  if (pool->in_flight && pool->ev) (void)hipEventSynchronize(pool->ev);
  for (PoolRequest* r : pool->active) {
    release(pool, r);
    delete r;
  }
  for (PoolRequest* r : pool->queue) delete r;
  for (auto& kv : pool->finished) delete kv.second;
  delete pool->engine;
  if (pool->capture) (void)hipStreamDestroy(pool->capture);
  if (pool->ev) (void)hipEventDestroy(pool->ev);
  if (pool->h_states) (void)hipHostFree(pool->h_states);
  if (pool->h_mats) (void)hipHostFree(pool->h_mats);
  delete pool;
  return QDWF_OK;
}

int qdwf_pool_submit(qdwf_pool* pool, const qdwf_request* req, uint64_t* id) {
  if (!pool || !req || !id) return fail(QDWF_EINVAL, "null argument");
  if (!req->U || !req->b || !req->x_out) return fail(QDWF_EINVAL, "request buffers must be set");
  const qdwf_solve_params& p = req->params;
  if (!validate_params(p)) return fail(QDWF_EINVAL, "tol must be in (0, 1) and delta in [0, 1)");
  if (p.inner_prec != pool->prm.inner_prec || p.layout != pool->prm.layout)
    return fail(QDWF_EINVAL, "the request's inner precision and layout must be the pool's");
  const qdwf_action& a = req->act;
  for (int mu = 0; mu < 4; ++mu)
    if (a.L[mu] < 2 || (a.L[mu] & 1) || (a.bc[mu] != 1 && a.bc[mu] != -1))
      return fail(QDWF_EINVAL, "bad lattice extent or boundary in direction %d", mu);
  if (a.Ls < 8 || a.Ls > 32) return fail(QDWF_EINVAL, "served solves take 8 <= Ls <= 32 (got %d)", a.Ls);
  const double al = a.b * (4.0 - a.M5) + 1.0;
  if (!(std::fabs(a.b) > 0.0) || !std::isfinite(al) || al == 0.0 || !std::isfinite(a.mf) ||
      !std::isfinite(a.c))
    return fail(QDWF_EINVAL, "degenerate action");
  const size_t need = request_total(a, p.inner_prec);
  const size_t room = pool->alloc.size - pool->overhead;
  if (need > room)
    return fail(QDWF_EINVAL, "request needs %zu bytes, more than the arena holds for requests (%zu)",
                need, room);
  PoolRequest* r = new (std::nothrow) PoolRequest();
  if (!r) return fail(QDWF_ENOMEM, "host allocation failed");
  r->id = pool->next_id++;
  r->act = a;
  r->prm = p;
  r->U = req->U;
  r->b = req->b;
  r->x_out = req->x_out;
  pool->queue.push_back(r);
  pool->where[r->id] = 0;
  *id = r->id;
  return QDWF_OK;
}

int qdwf_pool_step(qdwf_pool* pool, void* stream, int* n_active) {
  if (!pool) return fail(QDWF_EINVAL, "null pool");
  Dev dg(pool->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int rc;
  bool changed = false;
  // 1. the last round: retire what finished in it
  if (pool->in_flight) {
    QDWF_HIP(hipEventSynchronize(pool->ev));
    pool->in_flight = false;
    std::vector<PoolRequest*> still;
    for (PoolRequest* r : pool->active) {
      const RhsState& s = pool->h_states[r->slot];
      if (s.status == ST_RUN || s.status == ST_UPDATE) {
        still.push_back(r);
        continue;
      }
      r->stats.iterations = s.iters;
      r->stats.reliable_updates = s.ru;
      r->stats.converged = s.status == ST_DONE ? 1 : 0;
      r->stats.true_residual = s.bb > 0 ? std::sqrt(s.rr_true / s.bb) : 0.0;
      r->stats.flops = (int64_t)4 * (s.iters + s.ru + 1) * 1320 * r->ctx->g.n5h;
      r->stats.seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_admit).count();
      rc = launch_pack(r->ctx, r->x_out, QDWF_F64, pool->prm.layout, r->m.xo, QDWF_F64, QDWF_ODD, 1,
                       st, true);
      // the arena room is reused only by work queued after this unpack
      release(pool, r);
      finish(pool, r, rc ? rc : status_code(s.status));
      changed = true;
    }
    pool->active.swap(still);
  }
  // 2. admit from the head of the queue while the arena and the slots allow
  //    (first in, first out: a request that does not fit blocks the ones behind it)
  while (!pool->queue.empty() && (int)pool->active.size() < pool->max_slots) {
    PoolRequest* r = pool->queue.front();
    rc = admit(pool, r, st);
    if (rc == QDWF_EBUSY) break;
    pool->queue.pop_front();
    if (rc) {
      release(pool, r);
      finish(pool, r, rc);
      continue;
    }
    pool->active.push_back(r);
    pool->where[r->id] = 1;
    changed = true;
  }
  // 3. one round for every member
  if (changed) {
    std::vector<GroupMember> ms;
    for (PoolRequest* r : pool->active) ms.push_back(r->m);
    if ((rc = pool->engine->set_members(ms.data(), (int)ms.size(), st))) return rc;
  }
  if (!pool->active.empty()) {
    if ((rc = pool->engine->launch_round(st))) return rc;
    QDWF_HIP(hipMemcpyAsync(pool->h_states, pool->d_states, sizeof(RhsState) * pool->max_slots,
                            hipMemcpyDeviceToHost, st));
    QDWF_HIP(hipEventRecord(pool->ev, st));
    pool->in_flight = true;
  }
  if (n_active) *n_active = (int)pool->active.size();
  return QDWF_OK;
}

int qdwf_pool_poll(qdwf_pool* pool, uint64_t id, qdwf_solve_stats* stats) {
  if (!pool) return fail(QDWF_EINVAL, "null pool");
  auto w = pool->where.find(id);
  if (w == pool->where.end()) return fail(QDWF_EINVAL, "unknown request id %llu", (unsigned long long)id);
  if (w->second != 2) return QDWF_EBUSY;
  PoolRequest* r = pool->finished[id];
  if (stats) *stats = r->stats;
  const int rc = r->rc;
  pool->finished.erase(id);
  pool->where.erase(w);
  delete r;
  if (rc == QDWF_ENOTCONV) set_error("request %llu reached max_iter", (unsigned long long)id);
  return rc;
}

int qdwf_pool_info(qdwf_pool* pool, size_t* in_use, size_t* peak, int* n_active, int* n_queued) {
  if (!pool) return fail(QDWF_EINVAL, "null pool");
  if (in_use) *in_use = pool->alloc.used;
  if (peak) *peak = pool->peak;
  if (n_active) *n_active = (int)pool->active.size();
  if (n_queued) *n_queued = (int)pool->queue.size();
  return QDWF_OK;
}

}  // extern "C"
