// Autotuner for the hop kernel's launch shape and for the site traversal
// order and spinor layout.
//
// For a context, precision, layout and number of right-hand sides, every
// candidate shape -- threads per block, right-hand sides per block, XCD-aware
// block order on/off, and an LDS reservation that caps how many blocks share
// a CU -- is timed with HIP events on the full operator D and on D^dag, and
// the fastest is kept in the context. With QDWF_TUNE_CACHE naming a file, the
// results are appended there (one JSON object per line, keyed by lattice, Ls,
// precision, layout, dagger, nrhs and device architecture) and read back when
// a context of the same shape is created, so tuning happens once per machine.
//
// The traversal order (split and sweep dimension, tile) is fixed when a
// context is created, since the links and every packed field follow it, and
// the layout is the caller's choice when packing; qdwf_tune_traversal
// therefore times candidates on throwaway contexts (unit links, zero fields)
// and reports the fastest traversal and layout, which qdwf_create of the same
// lattice then takes from the cache.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

namespace qdwf {

namespace {

typedef std::tuple<int, int, int, int> TuneKey;   // prec, layout, dagger, nrhs

std::mutex g_mu;
std::map<const qdwf_ctx*, std::map<TuneKey, HopShape>> g_tuned;
std::map<const qdwf_ctx*, bool> g_loaded;   // cache file read for this context

std::string arch_name(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
  std::string s = p.gcnArchName;
  const size_t c = s.find(':');
  return c == std::string::npos ? s : s.substr(0, c);
}

std::string cache_key(const qdwf_ctx* c, int prec, int layout, int dagger, int nrhs) {
  char buf[256];
  snprintf(buf, sizeof(buf), "%dx%dx%dx%d_Ls%d_p%d_l%d_d%d_n%d_t%d.%d.%d.%d_o%d.%d_%s", c->g.L[0],
           c->g.L[1], c->g.L[2], c->g.L[3], c->g.Ls, prec, layout, dagger, nrhs, c->tile[0],
           c->tile[1], c->tile[2], c->tile[3], c->order[0], c->order[1], arch_name(c->device).c_str());
  return buf;
}

void cache_store(const std::string& key, const HopShape& s, double ms) {
  const char* path = std::getenv("QDWF_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"threads\": %d, \"nrb\": %d, \"xcd\": %d, \"lds_pad\": %d, \"sweep\": %d, \"ms\": %.6f}\n",
               key.c_str(), s.threads, s.nrb, s.xcd, s.lds_pad, s.sweep, ms);
  std::fclose(f);
}

bool cache_load(const std::string& key, HopShape* out) {
  const char* path = std::getenv("QDWF_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char k[256];
    HopShape s;
    double ms;
    if (std::sscanf(line, "{\"key\": \"%255[^\"]\", \"threads\": %d, \"nrb\": %d, \"xcd\": %d, \"lds_pad\": %d, \"sweep\": %d, \"ms\": %lf}",
                    k, &s.threads, &s.nrb, &s.xcd, &s.lds_pad, &s.sweep, &ms) == 7 &&
        key == k) {
      *out = s;   // the last entry for a key wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

std::string trav_key(const int L[4], int Ls, int device) {
  char buf[160];
  snprintf(buf, sizeof(buf), "trav_%dx%dx%dx%d_Ls%d_%s", L[0], L[1], L[2], L[3], Ls,
           arch_name(device).c_str());
  return buf;
}

void trav_store(const std::string& key, const Traversal& t, int layout, int prec, int nrhs,
                double ms) {
  const char* path = std::getenv("QDWF_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"split\": %d, \"sweep\": %d, \"tile\": [%d, %d, %d, %d], "
               "\"layout\": %d, \"prec\": %d, \"nrhs\": %d, \"ms\": %.6f}\n",
               key.c_str(), t.split, t.sweep, t.tile[0], t.tile[1], t.tile[2], t.tile[3], layout,
               prec, nrhs, ms);
  std::fclose(f);
}

bool trav_load(const std::string& key, Traversal* out) {
  const char* path = std::getenv("QDWF_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char k[160];
    Traversal t;
    if (std::sscanf(line, "{\"key\": \"%159[^\"]\", \"split\": %d, \"sweep\": %d, \"tile\": [%d, %d, %d, %d]",
                    k, &t.split, &t.sweep, &t.tile[0], &t.tile[1], &t.tile[2], &t.tile[3]) == 7 &&
        key == k && t.split >= 0 && t.split < 4 && t.sweep >= 0 && t.sweep < 4 &&
        t.split != t.sweep && t.tile[0] > 0 && t.tile[1] > 0 && t.tile[2] > 0 && t.tile[3] > 0) {
      *out = t;   // the last entry for a key wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

__global__ void unit_gauge_kernel(double* U, long n) {
  // canonical complex128 links, 9 complex entries per link: the identity
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ab = (int)(i % 9);
    U[2 * i] = (ab % 4 == 0) ? 1.0 : 0.0;
    U[2 * i + 1] = 0.0;
  }
}

}  // namespace

Traversal pick_traversal(const int L[4], int Ls, int device) {
  const char* eo = std::getenv("QDWF_ORDER");
  const char* et = std::getenv("QDWF_TILE");
  if ((eo && *eo) || (et && *et)) {
    int sd = 2, wd = 3;
    if (eo) {
      int a = -1, b = -1;
      if (std::sscanf(eo, "%d,%d", &a, &b) == 2 && a >= 0 && a < 4 && b >= 0 && b < 4 && a != b) {
        sd = a;
        wd = b;
      }
    }
    Traversal t = default_traversal(L, sd, wd);
    if (et) {
      int t4[4] = {0, 0, 0, 1};
      const int n = std::sscanf(et, "%d,%d,%d,%d", &t4[0], &t4[1], &t4[2], &t4[3]);
      if (n >= 3 && t4[0] > 0 && t4[1] > 0 && t4[2] > 0 && t4[3] > 0)
        for (int mu = 0; mu < 4; ++mu) t.tile[mu] = t4[mu];
      t.tile[wd] = 1;
    }
    return t;
  }
  Traversal t;
  if (Ls > 0) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (trav_load(trav_key(L, Ls, device), &t)) return t;
  }
  return default_traversal(L, 2, 3);
}

bool tuned_shape(const qdwf_ctx* ctx, int prec, int layout, int dagger, int nrhs, HopShape* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_loaded[ctx]) {
    // first use of this context: take every cached entry that matches it
    g_loaded[ctx] = true;
    const char* path = std::getenv("QDWF_TUNE_CACHE");
    if (path && *path)
    for (int p = QDWF_F64; p <= QDWF_BF16; ++p)
      for (int l = 0; l < 2; ++l)
        for (int d = 0; d < 2; ++d)
          for (int n : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32}) {
            HopShape s;
            if (cache_load(cache_key(ctx, p, l, d, n), &s)) g_tuned[ctx][TuneKey(p, l, d, n)] = s;
          }
  }
  auto it = g_tuned.find(ctx);
  if (it != g_tuned.end()) {
    auto jt = it->second.find(TuneKey(prec, layout, dagger, nrhs));
    if (jt != it->second.end()) {
      *out = jt->second;
      return true;
    }
  }
  return false;
}

void forget_tuning(const qdwf_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tuned.erase(ctx);
  g_loaded.erase(ctx);
}

}  // namespace qdwf

using namespace qdwf;

extern "C" {

int qdwf_tune(qdwf_ctx* ctx, int prec, int layout, int nrhs, void* ws, void* stream,
              double* best_ms) {
  if (!ctx || !ws) return fail(QDWF_EINVAL, "null argument");
  if (prec < QDWF_F64 || prec > QDWF_BF16) return fail(QDWF_EINVAL, "unknown precision %d", prec);
  if (layout != QDWF_RIRI && layout != QDWF_RRII) return fail(QDWF_EINVAL, "unknown layout %d", layout);
  if (nrhs < 1 || nrhs > 4096) return fail(QDWF_EINVAL, "nrhs out of range");
  if (!ctx->gauge_set) return fail(QDWF_EINVAL, "gauge field not set");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const long half = ctx->g.n5h * 24;
  const size_t field = (size_t)2 * half * nrhs * prec_bytes(prec);
  char* in = reinterpret_cast<char*>(ws);
  char* out = in + ((field + 255) & ~(size_t)255);
  QDWF_HIP(hipMemsetAsync(in, 0, field, st));
  const double al = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
  const double be = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
  const size_t bytes = prec_bytes(prec);
  HopArgs a = {};
  a.in[0] = in + half * bytes;
  a.in[1] = in;
  a.out[0] = out;
  a.out[1] = out + half * bytes;
  a.z[0] = in;
  a.z[1] = in + half * bytes;
  a.rs_in = a.rs_out = a.rs_z = 2 * half;
  a.par0 = 0;
  a.npar = 2;
  a.nrhs = nrhs;
  a.epi = 1;
  a.hop_scale = -0.5;
  a.alpha = al;
  a.beta = be;
  hipEvent_t e0, e1;
  QDWF_HIP(hipEventCreate(&e0));
  QDWF_HIP(hipEventCreate(&e1));
  const int gpw = 64 / ctx->g.Ls;
  const int reps = 5;
  for (int dagger = 0; dagger < 2; ++dagger) {
    HopShape best = default_shape(ctx, prec, nrhs);
    double best_t = 1e30;
    for (int waves = 1; waves <= 4; ++waves) {
      const int G = waves * gpw;
      if (G > 32 || G < 1) continue;
      for (int nrb = 1; nrb <= G; ++nrb) {
        if (G % nrb || nrb > nrhs || (nrb > 1 && G / nrb < 2)) continue;
        for (int xcd = 0; xcd < 2; ++xcd)
          for (int pad : {0, 24 * 1024, 44 * 1024}) {
            HopShape s = {64 * waves, nrb, xcd, pad, 0};
            // warm-up launch; shapes the kernel rejects (LDS) are skipped
            if (launch_hop(ctx, prec, layout, dagger, a, st, &s) != QDWF_OK) continue;
            QDWF_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) launch_hop(ctx, prec, layout, dagger, a, st, &s);
            QDWF_HIP(hipEventRecord(e1, st));
            QDWF_HIP(hipEventSynchronize(e1));
            float ms = 0;
            QDWF_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms / reps < best_t) {
              best_t = ms / reps;
              best = s;
            }
          }
      }
    }
    // the t-sweep serves the full operator wherever it applies; keep it when
    // it beats the best checkerboard shape (the other fields still serve
    // the launches it does not take)
    if (sweep_eligible(ctx, prec, layout, a)) {
      HopShape s = best;
      s.sweep = 1;
      if (launch_hop(ctx, prec, layout, dagger, a, st, &s) == QDWF_OK) {
        QDWF_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) launch_hop(ctx, prec, layout, dagger, a, st, &s);
        QDWF_HIP(hipEventRecord(e1, st));
        QDWF_HIP(hipEventSynchronize(e1));
        float ms = 0;
        QDWF_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms / reps < best_t) {
          best_t = ms / reps;
          best = s;
        }
      }
    }
    {
      std::lock_guard<std::mutex> lk(g_mu);
      g_tuned[ctx][TuneKey(prec, layout, dagger, nrhs)] = best;
    }
    cache_store(cache_key(ctx, prec, layout, dagger, nrhs), best, best_t);
    if (best_ms) best_ms[dagger] = best_t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  forget_graph(ctx);   // a solve's cached iterations used the previous shapes
  set_error("");
  if (prev >= 0) (void)hipSetDevice(prev);
  return QDWF_OK;
}

int qdwf_tune_traversal(const qdwf_action* act, int device, int prec, int nrhs, void* stream,
                        int32_t* choice7, double* best_ms) {
  if (!act || !choice7) return fail(QDWF_EINVAL, "null argument");
  if (prec < QDWF_F64 || prec > QDWF_BF16) return fail(QDWF_EINVAL, "unknown precision %d", prec);
  if (nrhs < 1 || nrhs > 4096) return fail(QDWF_EINVAL, "nrhs out of range");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(QDWF_EINVAL, "device %d not available (%d devices)", device, ndev);
  int prev = -1;
  (void)hipGetDevice(&prev);
  struct Restore {
    int d;
    ~Restore() { if (d >= 0) (void)hipSetDevice(d); }
  } restore{prev};
  // the buffers and launches below belong to `device`
  if (hipSetDevice(device) != hipSuccess) return fail(QDWF_EDEVICE, "hipSetDevice(%d) failed", device);
  // candidates: split z, sweep t with (x, y) tiles of 32 or 16 by 2, 4 or 8
  // (z tile Lz/8), and the default tiles of split y / sweep t and split t /
  // sweep z; duplicates after capping by the extents are dropped
  const int* L = act->L;
  std::vector<Traversal> cands;
  auto add = [&](Traversal t) {
    for (int mu = 0; mu < 4; ++mu) t.tile[mu] = std::max(1, std::min(t.tile[mu], L[mu]));
    t.tile[t.sweep] = 1;
    for (const Traversal& u : cands)
      if (u.split == t.split && u.sweep == t.sweep && std::equal(u.tile, u.tile + 4, t.tile)) return;
    cands.push_back(t);
  };
  add(default_traversal(L, 2, 3));
  for (int tx : {32, 16})
    for (int ty : {4, 2, 8}) {
      Traversal t = default_traversal(L, 2, 3);
      t.tile[0] = tx;
      t.tile[1] = ty;
      add(t);
    }
  add(default_traversal(L, 1, 3));
  add(default_traversal(L, 3, 2));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int reps = 5;
  double best_t = 1e30;
  Traversal best = cands[0];
  int best_layout = QDWF_RIRI;
  void* dU = nullptr;
  void* dbuf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = QDWF_OK;
  for (const Traversal& t : cands) {
    qdwf_ctx* c = nullptr;
    rc = create_context(act, device, &t, &c);
    if (rc) break;
    if (!dU) {
      // unit links (the timing does not depend on their values) and two
      // zero fields, allocated once on this device
      const long nlink = 4L * c->g.V * 9;
      const size_t field = (size_t)2 * c->g.n5h * 24 * nrhs * prec_bytes(prec);
      const size_t fal = (field + 255) & ~(size_t)255;
      hipError_t e = hipMalloc(&dU, (size_t)nlink * 16);
      if (e == hipSuccess) e = hipMalloc(&dbuf, 2 * fal);
      if (e == hipSuccess) e = hipMemsetAsync(dbuf, 0, 2 * fal, st);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(unit_gauge_kernel, dim3(1024), dim3(256), 0, st,
                           reinterpret_cast<double*>(dU), nlink);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipEventCreate(&e0);
      if (e == hipSuccess) e = hipEventCreate(&e1);
      if (e != hipSuccess) {
        qdwf_destroy(c);
        rc = fail(e == hipErrorOutOfMemory ? QDWF_ENOMEM : QDWF_EDEVICE,
                  "traversal tuning buffers: %s", hipGetErrorString(e));
        break;
      }
    }
    rc = qdwf_set_gauge(c, dU, QDWF_F64, stream);
    if (rc) {
      qdwf_destroy(c);
      break;
    }
    const size_t field = (size_t)2 * c->g.n5h * 24 * nrhs * prec_bytes(prec);
    char* in = reinterpret_cast<char*>(dbuf);
    char* out = in + ((field + 255) & ~(size_t)255);
    for (int layout : {QDWF_RIRI, QDWF_RRII}) {
      rc = qdwf_apply_D(c, out, in, 0, prec, layout, nrhs, stream);   // warm-up
      if (rc) break;
      hipError_t e = hipEventRecord(e0, st);
      for (int r = 0; r < reps && e == hipSuccess && rc == QDWF_OK; ++r)
        rc = qdwf_apply_D(c, out, in, 0, prec, layout, nrhs, stream);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) rc = fail(QDWF_EDEVICE, "traversal timing: %s", hipGetErrorString(e));
      if (rc) break;
      if (ms / reps < best_t) {
        best_t = ms / reps;
        best = t;
        best_layout = layout;
      }
    }
    qdwf_destroy(c);
    if (rc) break;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (dbuf) (void)hipFree(dbuf);
  if (dU) (void)hipFree(dU);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    trav_store(trav_key(L, act->Ls, device), best, best_layout, prec, nrhs, best_t);
  }
  choice7[0] = best.split;
  choice7[1] = best.sweep;
  for (int k = 0; k < 4; ++k) choice7[2 + k] = best.tile[k];
  choice7[6] = best_layout;
  if (best_ms) *best_ms = best_t;
  set_error("");
  return QDWF_OK;
}

int qdwf_traversal(qdwf_ctx* ctx, int32_t* order6) {
  if (!ctx || !order6) return fail(QDWF_EINVAL, "null argument");
  order6[0] = ctx->order[0];
  order6[1] = ctx->order[1];
  for (int k = 0; k < 4; ++k) order6[2 + k] = ctx->tile[k];
  return QDWF_OK;
}

int qdwf_tuned_shape(qdwf_ctx* ctx, int prec, int layout, int dagger, int nrhs, int32_t* shape4) {
  if (!ctx || !shape4) return fail(QDWF_EINVAL, "null argument");
  HopShape s;
  if (!tuned_shape(ctx, prec, layout, dagger, nrhs, &s)) s = default_shape(ctx, prec, nrhs);
  shape4[0] = s.threads;
  shape4[1] = s.nrb;
  shape4[2] = s.xcd;
  shape4[3] = s.lds_pad;
  return QDWF_OK;
}

}  // extern "C"
