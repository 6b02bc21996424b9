// Serving pool: continuous batching of domain-wall CG solves.
//
// Requests (each with its own lattice, Ls, mass, gauge field and source)
// wait in FIFO order until their device footprint fits the pool's HBM budget
// and a slot is free; then they are admitted: a context is created, the
// links and the source are packed, and a resumable mixed-precision solver is
// started on the slot's own stream. Every qdwf_pool_step advances each active
// request by one round (a batch of inner iterations or a reliable update) --
// all rounds are launched before any is waited for, so work from different
// requests overlaps on the device -- then retires the finished ones, writing
// their solution into the caller's buffer and freeing their memory, so the
// next step can admit more. A request's arithmetic depends only on its own
// data (its own reductions, its own round schedule), so its result is the
// same whether it runs alone or among others.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "common.h"
#include "solver.h"

namespace qdwf {

struct PoolRequest {
  uint64_t id;
  qdwf_action act;
  qdwf_solve_params prm;
  const void* U;
  const void* b;
  void* x_out;
  size_t bytes;
  // while admitted
  qdwf_ctx* ctx = nullptr;
  void* mem = nullptr;
  Solver* solver = nullptr;
  int slot = -1;
  // once finished
  int rc = QDWF_OK;
  qdwf_solve_stats stats = {};
  std::chrono::steady_clock::time_point t_admit;
};

}  // namespace qdwf

struct qdwf_pool {
  int device;
  size_t budget, in_use = 0, peak = 0;
  int max_slots;
  std::vector<hipStream_t> streams;
  std::vector<char> slot_busy;
  std::deque<qdwf::PoolRequest*> queue;
  std::vector<qdwf::PoolRequest*> active;
  std::map<uint64_t, qdwf::PoolRequest*> finished;
  std::map<uint64_t, int> where;   // 0 queued, 1 active, 2 finished
  uint64_t next_id = 1;
};

using namespace qdwf;

namespace {

size_t half_bytes(const qdwf_action& a) {
  return (size_t)a.L[0] * a.L[1] * a.L[2] * a.L[3] / 2 * a.Ls * 24 * 8;
}

size_t request_bytes(const qdwf_action& a, const qdwf_solve_params& p) {
  // context (tables, links in four precisions) + solver workspace + FP64 x_o and b_o
  return ctx_bytes(a) + solve_ws_bytes_for(a, p.inner_prec, 1) + 2 * half_bytes(a) + 1024;
}

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&prev) == hipSuccess) (void)hipSetDevice(d);
  }
  ~Dev() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

void release(qdwf_pool* pool, PoolRequest* r) {
  delete r->solver;
  r->solver = nullptr;
  if (r->mem) (void)hipFree(r->mem);
  r->mem = nullptr;
  if (r->ctx) qdwf_destroy(r->ctx);
  r->ctx = nullptr;
  if (r->slot >= 0) pool->slot_busy[r->slot] = 0;
  r->slot = -1;
  pool->in_use -= r->bytes;
}

int admit(qdwf_pool* pool, PoolRequest* r) {
  int slot = -1;
  for (int i = 0; i < pool->max_slots; ++i)
    if (!pool->slot_busy[i]) { slot = i; break; }
  if (slot < 0) return fail(QDWF_EBUSY, "no free slot");
  hipStream_t st = pool->streams[slot];
  int rc = qdwf_create(&r->act, pool->device, &r->ctx);
  if (rc) return rc;
  const size_t hb = half_bytes(r->act);
  const size_t ws = solve_ws_bytes_for(r->act, r->prm.inner_prec, 1);
  const size_t total = ws + 2 * hb + 512;
  if (hipMalloc(&r->mem, total) != hipSuccess) {
    qdwf_destroy(r->ctx);
    r->ctx = nullptr;
    return fail(QDWF_ENOMEM, "pool request allocation of %zu bytes failed", total);
  }
  r->slot = slot;
  pool->slot_busy[slot] = 1;
  pool->in_use += r->bytes;
  pool->peak = std::max(pool->peak, pool->in_use);
  char* m = reinterpret_cast<char*>(r->mem);
  double* xo = reinterpret_cast<double*>(m);
  double* bo = reinterpret_cast<double*>(m + hb);
  void* w = m + 2 * hb + 256 - ((uintptr_t)(m + 2 * hb) & 255);
  if ((rc = qdwf_set_gauge(r->ctx, r->U, QDWF_F64, st))) return rc;
  if ((rc = qdwf_pack_spinor(r->ctx, bo, QDWF_F64, r->prm.layout, r->b, QDWF_F64, QDWF_ODD, 1, st)))
    return rc;
  qdwf_solve_params p = r->prm;
  p.system = QDWF_SYS_NORMAL_PC;
  p.x0_is_guess = 0;
  r->solver = make_solver(r->ctx, p, 1, xo, bo, w, st);
  if (!r->solver) return fail(QDWF_EINVAL, "unknown inner precision");
  r->t_admit = std::chrono::steady_clock::now();
  return r->solver->begin();
}

}  // namespace

extern "C" {

size_t qdwf_request_bytes(const qdwf_action* act, const qdwf_solve_params* params) {
  if (!act || !params) return 0;
  return request_bytes(*act, *params);
}

int qdwf_pool_create(int device, size_t hbm_budget, int max_slots, qdwf_pool** out) {
  if (!out) return fail(QDWF_EINVAL, "null argument");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 64) return fail(QDWF_EINVAL, "max_slots %d out of [1, 64]", max_slots);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(QDWF_EINVAL, "device %d not available", device);
  Dev dg(device);
  qdwf_pool* p = new (std::nothrow) qdwf_pool();
  if (!p) return fail(QDWF_ENOMEM, "host allocation failed");
  p->device = device;
  p->budget = hbm_budget;
  p->max_slots = max_slots;
  p->slot_busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : p->streams) (void)hipStreamDestroy(t);
      delete p;
      return fail(QDWF_EDEVICE, "stream creation failed");
    }
    p->streams.push_back(s);
  }
  *out = p;
  return QDWF_OK;
}

int qdwf_pool_destroy(qdwf_pool* pool) {
  if (!pool) return QDWF_OK;
  Dev dg(pool->device);
  for (hipStream_t s : pool->streams) (void)hipStreamSynchronize(s);
  for (PoolRequest* r : pool->active) { release(pool, r); delete r; }
  for (PoolRequest* r : pool->queue) delete r;
  for (auto& kv : pool->finished) delete kv.second;
  for (hipStream_t s : pool->streams) (void)hipStreamDestroy(s);
  delete pool;
  return QDWF_OK;
}

int qdwf_pool_submit(qdwf_pool* pool, const qdwf_request* req, uint64_t* id) {
  if (!pool || !req || !id) return fail(QDWF_EINVAL, "null argument");
  if (!req->U || !req->b || !req->x_out) return fail(QDWF_EINVAL, "request buffers must be set");
  const qdwf_solve_params& p = req->params;
  if (!(p.tol > 0.0 && p.tol < 1.0)) return fail(QDWF_EINVAL, "tol must be in (0, 1)");
  if (p.inner_prec < QDWF_F64 || p.inner_prec > QDWF_BF16) return fail(QDWF_EINVAL, "inner precision");
  if (p.layout != QDWF_RIRI && p.layout != QDWF_RRII) return fail(QDWF_EINVAL, "layout");
  // validate the action the way qdwf_create will, without allocating
  for (int mu = 0; mu < 4; ++mu)
    if (req->act.L[mu] < 2 || (req->act.L[mu] & 1) || (req->act.bc[mu] != 1 && req->act.bc[mu] != -1))
      return fail(QDWF_EINVAL, "bad lattice extent or boundary in direction %d", mu);
  if (req->act.Ls < 2 || req->act.Ls > 64) return fail(QDWF_EINVAL, "Ls out of range");
  PoolRequest* r = new (std::nothrow) PoolRequest();
  if (!r) return fail(QDWF_ENOMEM, "host allocation failed");
  r->id = pool->next_id++;
  r->act = req->act;
  r->prm = p;
  r->U = req->U;
  r->b = req->b;
  r->x_out = req->x_out;
  r->bytes = request_bytes(req->act, p);
  if (r->bytes > pool->budget) {
    const size_t need = r->bytes;
    delete r;
    return fail(QDWF_EINVAL, "request needs %zu bytes, more than the pool budget %zu", need,
                pool->budget);
  }
  pool->queue.push_back(r);
  pool->where[r->id] = 0;
  *id = r->id;
  return QDWF_OK;
}

int qdwf_pool_step(qdwf_pool* pool, int* n_active) {
  if (!pool) return fail(QDWF_EINVAL, "null pool");
  Dev dg(pool->device);
  int rc;
  // 1. advance every request admitted in an earlier step by one round
  for (PoolRequest* r : pool->active)
    if ((rc = r->solver->launch())) return rc;
  // 2. admit from the head of the queue while the budget and slots allow
  //    (first in, first out: a request that does not fit blocks the ones behind it)
  std::vector<PoolRequest*> admitted;
  while (!pool->queue.empty() && (int)pool->active.size() + (int)admitted.size() < pool->max_slots) {
    PoolRequest* r = pool->queue.front();
    if (pool->in_use + r->bytes > pool->budget) break;
    pool->queue.pop_front();
    if ((rc = admit(pool, r))) {
      r->rc = rc;
      release(pool, r);
      pool->finished[r->id] = r;
      pool->where[r->id] = 2;
      continue;
    }
    admitted.push_back(r);
    pool->where[r->id] = 1;
  }
  for (PoolRequest* r : admitted) pool->active.push_back(r);
  // 3. wait for each request's round and retire the finished ones
  std::vector<PoolRequest*> still;
  for (PoolRequest* r : pool->active) {
    bool fin = false;
    if ((rc = r->solver->complete(&fin))) return rc;
    if (!fin) {
      still.push_back(r);
      continue;
    }
    r->rc = r->solver->result();
    r->solver->fill_stats(&r->stats);
    r->stats.seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - r->t_admit).count();
    hipStream_t st = pool->streams[r->slot];
    const double* xo = reinterpret_cast<const double*>(r->mem);
    if ((rc = qdwf_unpack_spinor(r->ctx, r->x_out, QDWF_F64, xo, QDWF_F64, r->prm.layout, QDWF_ODD, 1,
                                 st)))
      return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return fail(QDWF_EDEVICE, "stream sync failed");
    release(pool, r);
    pool->finished[r->id] = r;
    pool->where[r->id] = 2;
  }
  pool->active.swap(still);
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
  if (in_use) *in_use = pool->in_use;
  if (peak) *peak = pool->peak;
  if (n_active) *n_active = (int)pool->active.size();
  if (n_queued) *n_queued = (int)pool->queue.size();
  return QDWF_OK;
}

}  // extern "C"
