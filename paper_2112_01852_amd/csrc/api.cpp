// C ABI of libqdwf (declared in include/qdwf.h): argument validation, context
// lifecycle and dispatch to the HIP kernels. Nothing here allocates device
// memory outside qdwf_create / qdwf_set_gauge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <string>

#include "common.h"
#include "solver.h"

namespace qdwf {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

std::vector<double> build_local_matrices(const qdwf_action& a);

CtxLayout ctx_layout(const qdwf_action& a, bool with_geom, unsigned link_mask, bool derived) {
  Geom g;
  for (int mu = 0; mu < 4; ++mu) g.L[mu] = a.L[mu];
  g.Ls = a.Ls;
  g.V = a.L[0] * a.L[1] * a.L[2] * a.L[3];
  g.Vh = g.V / 2;
  g.n5h = (long)g.Vh * g.Ls;
  const size_t Vh = (size_t)g.Vh, V = (size_t)g.V;
  const size_t none = SIZE_MAX;
  CtxLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += (bytes + 255) & ~(size_t)255;
    return at;
  };
  L.nbr = L.site_lex = L.idx = none;
  if (with_geom) {
    L.nbr = take(sizeof(int32_t) * 2 * 8 * Vh);
    L.site_lex = take(sizeof(int32_t) * 2 * Vh);
    L.idx = take(sizeof(int32_t) * V);
  }
  L.geom_bytes = o;
  const size_t mats = (size_t)MAT_COUNT * 2 * a.Ls * a.Ls;
  L.mat64 = take(sizeof(double) * mats);
  L.mat32 = take(sizeof(float) * mats);
  const size_t link_reals = (size_t)2 * 4 * Vh * 18;
  for (int p = 0; p < 4; ++p) {
    L.links[p] = (link_mask >> p & 1u) ? take(link_reals * prec_bytes(p)) : none;
    L.dlinks[p] = L.wlinks[p] = none;
  }
  if (derived && sweep_geometry(g))
    for (int p = QDWF_F32; p <= QDWF_BF16; ++p)
      if (link_mask >> p & 1u) L.dlinks[p] = take(2 * link_reals * prec_bytes(p));
  if (derived && g.Ls == 1)   // FP64 and FP32: measured slower with 16-bit storage
    for (int p = QDWF_F64; p <= QDWF_F32; ++p)
      if (link_mask >> p & 1u) L.wlinks[p] = take((size_t)2 * 4 * 18 * Vh * prec_bytes(p));
  L.total = o;
  return L;
}

size_t ctx_bytes(const qdwf_action& a) { return ctx_layout(a, true, 0xFu, true).total; }

void place_arrays(qdwf_ctx* c, char* base, const CtxLayout& lay) {
  auto at = [&](size_t off) -> void* { return off == SIZE_MAX ? nullptr : base + off; };
  if (lay.nbr != SIZE_MAX) {
    c->d_nbr = reinterpret_cast<int32_t*>(at(lay.nbr));
    c->d_site_lex = reinterpret_cast<int32_t*>(at(lay.site_lex));
    c->d_idx = reinterpret_cast<int32_t*>(at(lay.idx));
  }
  c->d_mat64 = reinterpret_cast<double*>(at(lay.mat64));
  c->d_mat32 = reinterpret_cast<float*>(at(lay.mat32));
  for (int p = 0; p < 4; ++p) {
    c->d_links[p] = at(lay.links[p]);
    c->d_dlinks[p] = at(lay.dlinks[p]);
    c->d_wlinks[p] = at(lay.wlinks[p]);
  }
}

hipError_t upload_tables(qdwf_ctx* c, bool with_geom) {
  hipError_t e = hipSuccess;
  const GeomTables& G = *c->geo;
  if (with_geom) {
    e = hipMemcpy(c->d_nbr, G.nbr.data(), sizeof(int32_t) * G.nbr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->d_site_lex, G.site_lex.data(), sizeof(int32_t) * G.site_lex.size(),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->d_idx, G.idx.data(), sizeof(int32_t) * G.idx.size(), hipMemcpyHostToDevice);
  }
  const std::vector<float> m32(c->h_mat.begin(), c->h_mat.end());
  if (e == hipSuccess)
    e = hipMemcpy(c->d_mat64, c->h_mat.data(), sizeof(double) * c->h_mat.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->d_mat32, m32.data(), sizeof(float) * m32.size(), hipMemcpyHostToDevice);
  return e;
}

Traversal default_traversal(const int L[4], int sd, int wd) {
  Traversal t;
  t.split = sd;
  t.sweep = wd;
  if (sd == 2 && wd == 3) {
    t.tile[0] = std::min(L[0], 32);
    t.tile[1] = std::min(L[1], 4);
    t.tile[2] = std::max(1, L[2] / 8);
    t.tile[3] = 1;
  } else {
    for (int mu = 0; mu < 4; ++mu) t.tile[mu] = std::min(L[mu], 4);
    t.tile[sd] = std::max(1, L[sd] / 8);
  }
  t.tile[wd] = 1;
  return t;
}

std::shared_ptr<const GeomTables> build_geometry(const int L[4], const int bc[4],
                                                 const Traversal& tr) {
  auto G = std::make_shared<GeomTables>();
  const int V = L[0] * L[1] * L[2] * L[3], Vh = V / 2;
  for (int mu = 0; mu < 4; ++mu) { G->L[mu] = L[mu]; G->bc[mu] = bc[mu]; }
  // Internal site order of each parity. The lattice is cut into 8 slabs
  // along the split dimension, one per XCD (blocks of consecutive internal
  // sites reach the XCDs in contiguous ranges); inside a slab, tiles over the
  // other three dimensions are swept along the sweep dimension. The sites a
  // XCD works on at any moment then form a compact 4D region whose
  // neighbours are still in its L2, and all XCDs advance along the sweep
  // together, so neighbours shared across XCDs meet in the last-level cache.
  const int sd = tr.split, wd = tr.sweep;
  int tile[4];
  for (int mu = 0; mu < 4; ++mu) tile[mu] = std::max(1, tr.tile[mu]);
  tile[wd] = 1;
  for (int k = 0; k < 4; ++k) G->tile[k] = tile[k];
  G->order[0] = sd;
  G->order[1] = wd;
  std::vector<int64_t> key(V);
  for (int lex = 0; lex < V; ++lex) {
    int x[4], r = lex;
    for (int mu = 0; mu < 4; ++mu) { x[mu] = r % L[mu]; r /= L[mu]; }
    int64_t k = (x[sd] * 8) / L[sd];
    for (int mu = 3; mu >= 0; --mu)
      if (mu != wd) k = k * L[mu] + x[mu] / tile[mu];
    k = k * L[wd] + x[wd];
    for (int mu = 3; mu >= 0; --mu)
      if (mu != wd) k = k * L[mu] + x[mu] % tile[mu];
    key[lex] = k;
  }
  G->site_lex.assign((size_t)2 * Vh, 0);
  G->idx.assign((size_t)V, 0);
  {
    std::vector<int> order(V);
    for (int i = 0; i < V; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    int cnt[2] = {0, 0};
    for (int lex : order) {
      int x[4], r = lex;
      for (int mu = 0; mu < 4; ++mu) { x[mu] = r % L[mu]; r /= L[mu]; }
      const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
      const int i = cnt[p]++;
      G->site_lex[(size_t)p * Vh + i] = lex;
      G->idx[lex] = i;
    }
  }
  // neighbour and boundary tables in the internal order
  G->nbr.assign((size_t)2 * 8 * Vh, 0);
  G->sign.assign((size_t)2 * 8 * Vh, 0);
  for (int lex = 0; lex < V; ++lex) {
    int x[4], r = lex;
    for (int mu = 0; mu < 4; ++mu) { x[mu] = r % L[mu]; r /= L[mu]; }
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int i = G->idx[lex];
    for (int d = 0; d < 8; ++d) {
      const int mu = d & 3;
      int y[4] = {x[0], x[1], x[2], x[3]};
      int sg = 1;
      if (d < 4) {
        if (++y[mu] == L[mu]) { y[mu] = 0; sg = bc[mu]; }
      } else {
        if (--y[mu] < 0) { y[mu] = L[mu] - 1; sg = bc[mu]; }
      }
      const int yl = ((y[3] * L[2] + y[2]) * L[1] + y[1]) * L[0] + y[0];
      G->nbr[((size_t)p * 8 + d) * Vh + i] = G->idx[yl];
      G->sign[((size_t)p * 8 + d) * Vh + i] = (int8_t)sg;
    }
  }
  return G;
}

}  // namespace qdwf

using namespace qdwf;

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

#define CTX_CHECK(ctx)                                                    \
  do {                                                                    \
    if (!(ctx)) return fail(QDWF_EINVAL, "null context");                 \
  } while (0)

int check_prec(int prec) {
  if (prec < QDWF_F64 || prec > QDWF_BF16) return fail(QDWF_EINVAL, "unknown precision %d", prec);
  return QDWF_OK;
}
int check_layout(int layout) {
  if (layout != QDWF_RRII && layout != QDWF_RIRI) return fail(QDWF_EINVAL, "unknown layout %d", layout);
  return QDWF_OK;
}
int check_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 4096) return fail(QDWF_EINVAL, "nrhs %d out of range [1, 4096]", nrhs);
  return QDWF_OK;
}
int check_ptr(const void* p, const char* what) {
  if (!p) return fail(QDWF_EINVAL, "%s is NULL", what);
  return QDWF_OK;
}
int check_gauge(const qdwf_ctx* ctx) {
  if (!ctx->gauge_set) return fail(QDWF_EINVAL, "gauge field not set (call qdwf_set_gauge first)");
  return QDWF_OK;
}

#define TRY(x)                 \
  do {                         \
    int rc_ = (x);             \
    if (rc_) return rc_;       \
  } while (0)

}  // namespace

extern "C" {

const char* qdwf_last_error(void) { return g_err.c_str(); }

int qdwf_create(const qdwf_action* act, int device, qdwf_ctx** out) {
  return qdwf::create_context(act, device, nullptr, out);
}

}  // extern "C"

int qdwf::create_context(const qdwf_action* act, int device, const Traversal* tr, qdwf_ctx** out) {
  if (!act || !out) return fail(QDWF_EINVAL, "null argument");
  *out = nullptr;
  for (int mu = 0; mu < 4; ++mu) {
    if (act->L[mu] < 2 || (act->L[mu] & 1))
      return fail(QDWF_EINVAL, "L[%d] = %d must be even and >= 2", mu, act->L[mu]);
    if (act->bc[mu] != 1 && act->bc[mu] != -1)
      return fail(QDWF_EINVAL, "bc[%d] = %d must be +1 or -1", mu, act->bc[mu]);
  }
  if (act->Ls < 1 || act->Ls > 64) return fail(QDWF_EINVAL, "Ls = %d must be in [1, 64]", act->Ls);
  if (act->Ls == 1 && ((long)act->L[0] * act->L[1] * act->L[2] * act->L[3] / 2) % 16 != 0)
    return fail(QDWF_EINVAL, "4D fields (Ls = 1) need a multiple of 16 sites per parity");
  const double V = (double)act->L[0] * act->L[1] * act->L[2] * act->L[3];
  if (V * act->Ls / 2 * 24 > 9.0e18 || V > 2.0e9) return fail(QDWF_EINVAL, "lattice too large");
  if (!(std::fabs(act->b) > 0.0) || !std::isfinite(act->b))
    return fail(QDWF_EINVAL, "Mobius b = %g must be finite and nonzero", act->b);
  const double al = act->b * (4.0 - act->M5) + 1.0;
  if (!std::isfinite(al) || al == 0.0 || !std::isfinite(act->mf) || !std::isfinite(act->c))
    return fail(QDWF_EINVAL, "degenerate action: alpha = b(4-M5)+1 = %g", al);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(QDWF_EINVAL, "device %d not available (%d devices)", device, ndev);
  DeviceGuard dg(device);
  if (!dg.ok) return fail(QDWF_EDEVICE, "hipSetDevice(%d) failed", device);

  qdwf_ctx* c = new (std::nothrow) qdwf_ctx();
  if (!c) return fail(QDWF_ENOMEM, "host allocation failed");
  c->act = *act;
  c->device = device;
  Geom& g = c->g;
  for (int mu = 0; mu < 4; ++mu) g.L[mu] = act->L[mu];
  g.Ls = act->Ls;
  g.V = act->L[0] * act->L[1] * act->L[2] * act->L[3];
  g.Vh = g.V / 2;
  g.n5h = (long)g.Vh * g.Ls;
  try {
    c->geo = build_geometry(act->L, act->bc, tr ? *tr : pick_traversal(act->L, act->Ls, device));
    c->h_mat = build_local_matrices(*act);
  } catch (const std::bad_alloc&) {
    delete c;
    return fail(QDWF_ENOMEM, "host allocation of the site tables failed");
  }
  for (int k = 0; k < 4; ++k) c->tile[k] = c->geo->tile[k];
  for (int k = 0; k < 2; ++k) c->order[k] = c->geo->order[k];
  // one device block holds every array of the context (its size is ctx_bytes)
  const CtxLayout lay = ctx_layout(*act, true, 0xFu, true);
  hipError_t e = hipMalloc(&c->d_block, lay.total);
  if (e != hipSuccess) {
    const int code = (e == hipErrorOutOfMemory) ? QDWF_ENOMEM : QDWF_EDEVICE;
    c->d_block = nullptr;
    qdwf_destroy(c);
    return fail(code, "device allocation of %zu bytes in qdwf_create failed: %s", lay.total,
                hipGetErrorString(e));
  }
  place_arrays(c, reinterpret_cast<char*>(c->d_block), lay);
  e = upload_tables(c, true);
  if (e != hipSuccess) {
    qdwf_destroy(c);
    return fail(QDWF_EDEVICE, "upload of the site tables failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return QDWF_OK;
}

extern "C" {

int qdwf_destroy(qdwf_ctx* ctx) {
  if (!ctx) return QDWF_OK;
  forget_tuning(ctx);
  forget_solver_state(ctx);
  DeviceGuard dg(ctx->device);
  if (ctx->d_block) (void)hipFree(ctx->d_block);
  delete ctx;
  return QDWF_OK;
}

int qdwf_set_gauge(qdwf_ctx* ctx, const void* U, int canon_prec, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(U, "U"));
  if (canon_prec != QDWF_F64 && canon_prec != QDWF_F32)
    return fail(QDWF_EINVAL, "canon_prec must be QDWF_F64 or QDWF_F32");
  DeviceGuard dg(ctx->device);
  TRY(launch_pack_links(ctx, U, canon_prec, S(stream)));
  TRY(launch_doubled_links(ctx, S(stream)));
  TRY(launch_wilson_links(ctx, S(stream)));
  ctx->gauge_set = true;
  return QDWF_OK;
}

size_t qdwf_field_reals(const qdwf_ctx* ctx, int subset) {
  if (!ctx) return 0;
  return (size_t)(subset == QDWF_FULL ? 2 : 1) * ctx->g.n5h * 24;
}

static int check_subset(int subset) {
  if (subset != QDWF_EVEN && subset != QDWF_ODD && subset != QDWF_FULL)
    return fail(QDWF_EINVAL, "unknown subset %d", subset);
  return QDWF_OK;
}

int qdwf_pack_spinor(qdwf_ctx* ctx, void* dst, int prec, int layout, const void* src,
                     int src_prec, int subset, int nrhs, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(dst, "dst"));
  TRY(check_ptr(src, "src"));
  TRY(check_prec(prec));
  TRY(check_layout(layout));
  TRY(check_subset(subset));
  TRY(check_nrhs(nrhs));
  DeviceGuard dg(ctx->device);
  return launch_pack(ctx, dst, prec, layout, src, src_prec, subset, nrhs, S(stream), false);
}

int qdwf_unpack_spinor(qdwf_ctx* ctx, void* dst, int dst_prec, const void* src, int prec,
                       int layout, int subset, int nrhs, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(dst, "dst"));
  TRY(check_ptr(src, "src"));
  TRY(check_prec(prec));
  TRY(check_layout(layout));
  TRY(check_subset(subset));
  TRY(check_nrhs(nrhs));
  DeviceGuard dg(ctx->device);
  return launch_pack(ctx, dst, prec, layout, src, dst_prec, subset, nrhs, S(stream), true);
}

static int common_checks(qdwf_ctx* ctx, const void* out, const void* in, int prec, int layout,
                         int nrhs) {
  CTX_CHECK(ctx);
  TRY(check_ptr(out, "out"));
  TRY(check_ptr(in, "in"));
  TRY(check_prec(prec));
  TRY(check_layout(layout));
  TRY(check_nrhs(nrhs));
  TRY(check_gauge(ctx));
  return QDWF_OK;
}

static double alpha_of(const qdwf_ctx* c) { return c->act.b * (4.0 - c->act.M5) + 1.0; }
static double beta_of(const qdwf_ctx* c) { return c->act.c * (4.0 - c->act.M5) - 1.0; }

int qdwf_apply_D(qdwf_ctx* ctx, void* out, const void* in, int dagger, int prec, int layout,
                 int nrhs, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  const size_t bytes = prec_bytes(prec);
  const long half = ctx->g.n5h * 24;
  const char* ib = reinterpret_cast<const char*>(in);
  char* ob = reinterpret_cast<char*>(out);
  HopArgs a = {};
  a.in[0] = ib + half * bytes;   // output even reads odd input
  a.in[1] = ib;
  a.out[0] = ob;
  a.out[1] = ob + half * bytes;
  a.z[0] = ib;
  a.z[1] = ib + half * bytes;
  a.rs_in = a.rs_out = a.rs_z = 2 * half;
  a.par0 = 0;
  a.npar = 2;
  a.nrhs = nrhs;
  a.epi = 1;
  a.hop_scale = -0.5;
  a.alpha = alpha_of(ctx);
  a.beta = beta_of(ctx);
  return launch_hop(ctx, prec, layout, dagger ? 1 : 0, a, S(stream));
}

int qdwf_apply_Dh(qdwf_ctx* ctx, void* out, const void* in, int subset, int dagger, int prec,
                  int layout, int nrhs, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  if (subset != QDWF_EVEN && subset != QDWF_ODD && subset != QDWF_FULL)
    return fail(QDWF_EINVAL, "subset must be 0, 1 or 2");
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  const long half = ctx->g.n5h * 24;
  const size_t bytes = prec_bytes(prec);
  const char* ib = reinterpret_cast<const char*>(in);
  char* ob = reinterpret_cast<char*>(out);
  HopArgs a = {};
  if (subset == QDWF_FULL) {
    a.in[0] = ib + half * bytes;   // output even reads odd input
    a.in[1] = ib;
    a.out[0] = ob;
    a.out[1] = ob + half * bytes;
    a.rs_in = a.rs_out = 2 * half;
    a.par0 = 0;
    a.npar = 2;
  } else {
    a.in[subset] = ib;             // half field of the other parity
    a.out[subset] = ob;
    a.rs_in = a.rs_out = half;
    a.par0 = subset;
    a.npar = 1;
  }
  a.nrhs = nrhs;
  a.epi = 0;
  a.hop_scale = 1.0;
  return launch_wilson(ctx, prec, layout, dagger ? 1 : 0, a, S(stream));
}

int qdwf_apply_Dw(qdwf_ctx* ctx, void* out, const void* in, double mass, int dagger, int prec,
                  int layout, int nrhs, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  if (!std::isfinite(mass)) return fail(QDWF_EINVAL, "mass must be finite");
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  const long half = ctx->g.n5h * 24;
  const size_t bytes = prec_bytes(prec);
  const char* ib = reinterpret_cast<const char*>(in);
  char* ob = reinterpret_cast<char*>(out);
  HopArgs a = {};
  a.in[0] = ib + half * bytes;
  a.in[1] = ib;
  a.out[0] = ob;
  a.out[1] = ob + half * bytes;
  a.z[0] = ib;
  a.z[1] = ib + half * bytes;
  a.rs_in = a.rs_out = a.rs_z = 2 * half;
  a.par0 = 0;
  a.npar = 2;
  a.nrhs = nrhs;
  a.epi = 1;
  a.hop_scale = -0.5;
  a.alpha = 4.0 + mass;
  return launch_wilson(ctx, prec, layout, dagger ? 1 : 0, a, S(stream));
}

int qdwf_su3_mul(void* C, const void* A, const void* B, int64_t n, int prec, int device,
                 void* stream) {
  if (n < 0) return fail(QDWF_EINVAL, "n must be >= 0");
  if (prec != QDWF_F64 && prec != QDWF_F32) return fail(QDWF_EINVAL, "precision must be F64 or F32");
  if (n > 0) {
    TRY(check_ptr(C, "C"));
    TRY(check_ptr(A, "A"));
    TRY(check_ptr(B, "B"));
    if (C == A || C == B) return fail(QDWF_EINVAL, "C must not alias A or B");
  }
  DeviceGuard dg(device);
  return launch_su3_mul(C, A, B, (long)n, prec, S(stream));
}

int qdwf_triad(void* a, const void* b, const void* c, double s, int64_t n, int prec, int device,
               void* stream) {
  if (n < 0) return fail(QDWF_EINVAL, "n must be >= 0");
  if (prec != QDWF_F64 && prec != QDWF_F32) return fail(QDWF_EINVAL, "precision must be F64 or F32");
  if (!std::isfinite(s)) return fail(QDWF_EINVAL, "s must be finite");
  if (n > 0) {
    TRY(check_ptr(a, "a"));
    TRY(check_ptr(b, "b"));
    TRY(check_ptr(c, "c"));
  }
  DeviceGuard dg(device);
  return launch_triad(a, b, c, s, (long)n, prec, S(stream));
}

int qdwf_apply_Mee(qdwf_ctx* ctx, void* out, const void* in, int subset, int dagger, int which,
                   int prec, int layout, int nrhs, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(out, "out"));
  TRY(check_ptr(in, "in"));
  TRY(check_prec(prec));
  TRY(check_layout(layout));
  TRY(check_nrhs(nrhs));
  TRY(check_subset(subset));
  if (which != QDWF_MEE_FWD && which != QDWF_MEE_INV) return fail(QDWF_EINVAL, "unknown operator %d", which);
  DeviceGuard dg(ctx->device);
  const long half = ctx->g.n5h * 24;
  const int nh = subset == QDWF_FULL ? 2 : 1;
  MatKind k = which == QDWF_MEE_FWD ? (dagger ? MAT_MEE_DAG : MAT_MEE)
                                    : (dagger ? MAT_MEEINV_DAG : MAT_MEEINV);
  return launch_local(ctx, prec, layout, k, out, in, nh, half, half * nh, nrhs, S(stream));
}

int qdwf_apply_Deo(qdwf_ctx* ctx, void* out, const void* in, int out_parity, int dagger,
                   int prec, int layout, int nrhs, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  if (out_parity != QDWF_EVEN && out_parity != QDWF_ODD) return fail(QDWF_EINVAL, "out_parity must be 0 or 1");
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  return apply_hop_parity(ctx, prec, layout, dagger ? 1 : 0, out_parity, out, in, nullptr, -0.5,
                          nrhs, ctx->g.n5h * 24, S(stream));
}

size_t qdwf_workspace_bytes(const qdwf_ctx* ctx, int op, int prec, int nrhs) {
  if (!ctx || nrhs < 1 || prec < QDWF_F64 || prec > QDWF_BF16) return 0;
  const size_t half = (size_t)ctx->g.n5h * 24 * prec_bytes(prec) * nrhs;
  const size_t al = (half + 255) & ~(size_t)255;
  switch (op) {
    case QDWF_OP_MPC: return 2 * al;
    case QDWF_OP_MDAGM: return 3 * al;
    case QDWF_OP_SOLVE: return solve_ws_bytes(ctx, prec, nrhs, 0);
    case QDWF_OP_REDUCE: return dot_ws_bytes((long)ctx->g.n5h * 24 * 2, nrhs);
    case QDWF_OP_TUNE: return 2 * ((2 * half + 255) & ~(size_t)255);
  }
  return 0;
}

int qdwf_apply_Mpc(qdwf_ctx* ctx, void* out, const void* in, int dagger, int prec, int layout,
                   int nrhs, void* ws, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  TRY(check_ptr(ws, "ws"));
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  const size_t half = (size_t)ctx->g.n5h * 24 * prec_bytes(prec) * nrhs;
  const size_t al = (half + 255) & ~(size_t)255;
  char* w = reinterpret_cast<char*>(ws);
  return apply_mpc(ctx, prec, layout, dagger ? 1 : 0, out, in, w, w + al, nrhs,
                   ctx->g.n5h * 24, S(stream));
}

int qdwf_apply_MdagM(qdwf_ctx* ctx, void* out, const void* in, int prec, int layout, int nrhs,
                     void* ws, void* stream) {
  TRY(common_checks(ctx, out, in, prec, layout, nrhs));
  TRY(check_ptr(ws, "ws"));
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  DeviceGuard dg(ctx->device);
  const size_t half = (size_t)ctx->g.n5h * 24 * prec_bytes(prec) * nrhs;
  const size_t al = (half + 255) & ~(size_t)255;
  char* w = reinterpret_cast<char*>(ws);
  return apply_mdagm(ctx, prec, layout, out, in, w, w + al, w + 2 * al, nrhs, ctx->g.n5h * 24,
                     S(stream));
}

int qdwf_dot(qdwf_ctx* ctx, double* out, const void* x, const void* y, int subset, int prec,
             int layout, int nrhs, void* ws, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(out, "out"));
  TRY(check_ptr(x, "x"));
  TRY(check_ptr(y, "y"));
  TRY(check_ptr(ws, "ws"));
  TRY(check_prec(prec));
  TRY(check_layout(layout));
  TRY(check_subset(subset));
  TRY(check_nrhs(nrhs));
  DeviceGuard dg(ctx->device);
  const long n = (long)(subset == QDWF_FULL ? 2 : 1) * ctx->g.n5h * 24;
  return dot_re_im(ctx, out, x, y, n, prec, layout, nrhs, ws, S(stream));
}

int qdwf_solve(qdwf_ctx* ctx, void* x, const void* b, int nrhs, const qdwf_solve_params* params,
               qdwf_solve_stats* stats, void* ws, void* stream) {
  CTX_CHECK(ctx);
  TRY(check_ptr(x, "x"));
  TRY(check_ptr(b, "b"));
  TRY(check_ptr(params, "params"));
  TRY(check_ptr(ws, "ws"));
  TRY(check_nrhs(nrhs));
  TRY(check_gauge(ctx));
  qdwf_solve_params p = *params;
  TRY(check_prec(p.inner_prec));
  TRY(check_layout(p.layout));
  if (p.system != QDWF_SYS_NORMAL_PC && p.system != QDWF_SYS_FULL)
    return fail(QDWF_EINVAL, "unknown system %d", p.system);
  if (!(p.tol > 0.0) || !(p.tol < 1.0)) return fail(QDWF_EINVAL, "tol must be in (0, 1)");
  if (p.delta < 0.0 || p.delta >= 1.0) return fail(QDWF_EINVAL, "delta must be in [0, 1)");
  if (p.check_every < 0 || p.check_every > 4096) return fail(QDWF_EINVAL, "check_every out of range");
  if (x == b) return fail(QDWF_EINVAL, "x must not alias b");
  DeviceGuard dg(ctx->device);
  qdwf_solve_stats local = {};
  qdwf_solve_stats* sp = stats ? stats : &local;
  std::memset(sp, 0, sizeof(*sp));
  const auto t0 = std::chrono::steady_clock::now();
  // graphs cannot be captured on the null stream: run such a call on a
  // private stream (the call is synchronous either way)
  hipStream_t run = S(stream);
  hipStream_t own = nullptr;
  if (p.use_graph && run == nullptr) {
    if (hipStreamSynchronize(nullptr) != hipSuccess ||
        hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess)
      return fail(QDWF_EDEVICE, "could not create a stream for graph capture");
    run = own;
  }
  const int rc = solve(ctx, reinterpret_cast<double*>(x), reinterpret_cast<const double*>(b), nrhs,
                       p, sp, ws, run);
  (void)hipStreamSynchronize(run);
  if (own) (void)hipStreamDestroy(own);
  sp->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc == QDWF_ENOTCONV) set_error("solver reached max_iter = %d before tol", p.max_iter);
  if (rc == QDWF_ENAN) set_error("solver met NaN/Inf or a breakdown (p^dag A p <= 0)");
  return rc;
}

int qdwf_geometry_tables(qdwf_ctx* ctx, int32_t* cb_of_lex, int32_t* nbr, int8_t* sign) {
  CTX_CHECK(ctx);
  const Geom& g = ctx->g;
  if (cb_of_lex)
    for (int l = 0; l < g.V; ++l) cb_of_lex[l] = ctx->geo->idx[l];
  // the kernels read [p][d][cb]; the exported order is [p][cb][d]
  if (nbr) {
    std::vector<int32_t> dev((size_t)2 * 8 * g.Vh);
    DeviceGuard dg(ctx->device);
    if (hipMemcpy(dev.data(), ctx->d_nbr, sizeof(int32_t) * dev.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(QDWF_EDEVICE, "copy of the neighbour table failed");
    for (int p = 0; p < 2; ++p)
      for (int cb = 0; cb < g.Vh; ++cb)
        for (int d = 0; d < 8; ++d) nbr[((size_t)p * g.Vh + cb) * 8 + d] = dev[((size_t)p * 8 + d) * g.Vh + cb];
  }
  if (sign)
    for (int p = 0; p < 2; ++p)
      for (int cb = 0; cb < g.Vh; ++cb)
        for (int d = 0; d < 8; ++d)
          sign[((size_t)p * g.Vh + cb) * 8 + d] = ctx->geo->sign[((size_t)p * 8 + d) * g.Vh + cb];
  return QDWF_OK;
}

}  // extern "C"
