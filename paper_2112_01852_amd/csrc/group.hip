// Grouped CG over many independent solves: descriptor tables, the grouped
// kernels (grid-stride walks over the units of every member, each unit one
// block of the single-solve kernels' work) and the captured round.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <type_traits>

#include "cgbody.h"
#include "group.h"
#include "hopbody.h"
#include "localbody.h"

namespace qdwf {

namespace {

constexpr int kHopGrid = 2048;     // blocks of a grouped hop launch (256 threads)
constexpr int kLocalThreads = 128;
constexpr int kLocalGrid = 1024;
constexpr int kBlasGrid = 2048;    // blocks of a grouped vector launch (RT threads)
constexpr int kLsMin = 8, kLsMax = 32;   // Ls a group accepts

// Units of one kind of grouped launch: member j owns [start[j], start[j+1]).
struct UnitHdr {
  int n;
  int start[kGroupMax + 1];
};

// A member's vectors and scalars as the grouped vector kernels see them.
struct GReq {
  RhsState* st;
  long n;                 // reals of a half field
  int NB;                 // reduction blocks
  int NBs;                // blocks of the reduction of the per-site sums
  long nsite;             // checkerboard sites (per-site sums of the fused CG step)
  double* site;           // per-site sums, written by the fused hops
  int vec_s, vec_r;       // the inner vectors may be walked in aligned words
  int vec_b;              // the FP64 source may be walked in aligned words
  int scale;              // inner vectors kept at unit RMS (inner precision below FP64)
  int max_iter;
  void* xl;               // inner solution increment (R)
  void* rl;               // inner residual (ResidStore of S)
  void* p;                // search direction (S)
  void* ap;               // output of M_pc^dag M_pc, which the fused step never stores
  double* xh;             // FP64 solution
  const double* b;        // FP64 source
  double* rh;             // FP64 true residual
  double* ax;             // FP64 M_pc^dag M_pc x
  double* part;           // reduction partials
  double tol2, delta2;
};

// M_ee^-1 (or M_ee^-dag) of a member with Ls != 16, between the hop stages.
struct GLoc {
  const void* in;
  void* out;
  const void* K;          // [2][Ls][Ls] in the compute type
  int Vh, Ls;
  long plane;
};

struct Table {
  UnitHdr blas, one, hop16, hopg, loc, sites;   // hop16: Ls = 16 members, hopg: the others
  GReq req[kGroupMax];
  HopK hop_s[4][kGroupMax];   // M_pc^dag M_pc stages in the inner precision
  HopK hop_d[4][kGroupMax];   // the same in FP64 (reliable updates)
  GLoc loc_s[2][kGroupMax];   // after stages 1 and 3, inner precision
  GLoc loc_d[2][kGroupMax];
};

__device__ inline int member_of(const UnitHdr& h, int u) {
  // largest j with start[j] <= u (members without units are skipped over)
  int lo = 0, hi = h.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (h.start[mid] <= u) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- grouped kernels ---------------------------------------------------------
// Hop stage `stage` (0..3) of M_pc^dag M_pc for the members whose status is
// `want`; FP64: the reliable update's operator. DPP16: the members with
// Ls = 16 (slices in DPP rows; MINV fuses M_ee^-1 into stages 0 and 2), else
// the other members (cross-lane permutes; stages 0 and 2 write te1 for
// g_local). One kernel per form: a kernel holding both bodies runs out of
// registers.
// Waves per SIMD the grouped hop's registers are planned for, so that no
// form spills: FP64 two on DPP rows in the interleaved layout (253-256
// registers) and one otherwise (its permute form needs more than the 256
// registers two waves leave; FP64 runs only in the reliable updates and in
// plain FP64 pools), the
// permute form of 16-bit storage three in the interleaved layout (144-162
// registers) and two in the split one, FP32 interleaved three (all grouped
// hops are one-parity ones), the others as the single-context hop.
template <class S, int LAYOUT, bool DPP16> struct GroupWaves {
  static constexpr int v =
      sizeof(S) == 8 ? ((DPP16 && LAYOUT == QDWF_RIRI) ? 2 : 1)
      : (sizeof(S) == 2 && !DPP16) ? (LAYOUT == QDWF_RIRI ? 3 : 2)
      : (std::is_same<S, float>::value && LAYOUT == QDWF_RIRI) ? 3
      : WavesPerEU<S, LAYOUT, DPP16>::v;
};

template <class S, int LAYOUT, bool DAG, bool DPP16, bool MINV, bool CHI>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(GroupWaves<S, LAYOUT, DPP16>::v, GroupWaves<S, LAYOUT, DPP16>::v)))
g_hop(const Table* __restrict__ t, int stage, int fp64, int want) {
  extern __shared__ __align__(16) unsigned char smem[];
  const UnitHdr& h = DPP16 ? t->hop16 : t->hopg;
  const int total = h.start[h.n];
  const HopK* tab = fp64 ? t->hop_d[stage] : t->hop_s[stage];
  for (int u = blockIdx.x; u < total; u += gridDim.x) {
    const int j = member_of(h, u);
    if (t->req[j].st->status != want) continue;
    hop_block<S, LAYOUT, DAG, DPP16, MINV, CHI>(tab[j], u - h.start[j], smem);
    __syncthreads();
  }
}

template <class S, int LAYOUT>
__global__ void __launch_bounds__(kLocalThreads)
g_local(const Table* __restrict__ t, int which, int fp64, int want) {
  typedef typename Store<S>::compute T;
  extern __shared__ __align__(16) unsigned char smem[];
  const UnitHdr& h = t->loc;
  const int total = h.start[h.n];
  const GLoc* tab = fp64 ? t->loc_d[which] : t->loc_s[which];
  for (int u = blockIdx.x; u < total; u += gridDim.x) {
    const int j = member_of(h, u);
    if (t->req[j].st->status != want) continue;
    const GLoc& l = tab[j];
    local_block<S, LAYOUT>(reinterpret_cast<const S*>(l.in), reinterpret_cast<S*>(l.out),
                           reinterpret_cast<const T*>(l.K), l.Vh, l.Ls, l.plane, u - h.start[j],
                           smem);
    __syncthreads();
  }
}

#define GROUP_LOOP(HDR)                                       \
  const UnitHdr& h = t->HDR;                                  \
  const int total = h.start[h.n];                             \
  for (int u = blockIdx.x; u < total; u += gridDim.x) {       \
    const int j = member_of(h, u);                            \
    const GReq& r = t->req[j];                                \
    const int bx = u - h.start[j];

// The fused iteration's reductions of the per-site sums (|M_pc p|^2, then
// |r|^2), alpha and beta as in the single-context solver, and the p pass
// (x takes its step in the last hop of M_pc^dag).
__global__ void __launch_bounds__(RT) g_sum_sites(const Table* __restrict__ t) {
  __shared__ double sh[RT];
  GROUP_LOOP(sites)
    if (r.st->status != ST_RUN) continue;
    k_sum_body(r.site, r.nsite, r.part, bx, r.NBs, 0, sh);
  }
}

__global__ void __launch_bounds__(RT) g_alpha(const Table* __restrict__ t) {
  __shared__ double sh[RT];
  for (int j = blockIdx.x; j < t->one.n; j += gridDim.x) {
    const GReq& r = t->req[j];
    k_alpha_body(r.part, r.NBs, r.st, 0, sh);
  }
}

__global__ void __launch_bounds__(RT) g_beta(const Table* __restrict__ t) {
  __shared__ double sh[RT];
  for (int j = blockIdx.x; j < t->one.n; j += gridDim.x) {
    const GReq& r = t->req[j];
    k_beta_body(r.part, r.NBs, r.st, r.delta2, 0, sh);
  }
}

// p = r + beta p in place while the member keeps running (its x took the
// iteration's step in the last hop of M_pc^dag)
template <class S>
__global__ void __launch_bounds__(RT) g_update_p(const Table* __restrict__ t) {
  typedef typename ResidStore<S>::t RR;
  GROUP_LOOP(blas)
    k_grp_p_body<RR, S>(reinterpret_cast<const RR*>(r.rl), reinterpret_cast<S*>(r.p), 0, 0, r.n,
                        r.n, r.st, r.vec_s && r.vec_r, bx, r.NB, 0);
  }
}

template <class R>
__global__ void __launch_bounds__(RT) g_fold_x(const Table* __restrict__ t) {
  GROUP_LOOP(blas)
    k_fold_x_body<R>(r.xh, reinterpret_cast<R*>(r.xl), r.n, r.n, r.n, r.st, bx, r.NB, 0, nullptr);
  }
}

__global__ void __launch_bounds__(RT) g_resid(const Table* __restrict__ t) {
  __shared__ double sh[RT];
  GROUP_LOOP(blas)
    if (r.st->status != ST_UPDATE) continue;
    k_resid_body(r.b, r.ax, r.rh, r.n, r.n, r.n, r.part, bx, r.NB, 0, sh);
  }
}

__global__ void __launch_bounds__(RT) g_ru_decide(const Table* __restrict__ t) {
  __shared__ double sh[RT];
  for (int j = blockIdx.x; j < t->one.n; j += gridDim.x) {
    const GReq& r = t->req[j];
    const int first = r.st->first;
    __syncthreads();   // every thread has read `first` before the body may clear it
    k_ru_decide_body(r.part, r.NB, r.st, r.tol2, (double)r.n, r.scale, first, 0, sh);
  }
}

template <class S, class R>
__global__ void __launch_bounds__(RT) g_ru_apply(const Table* __restrict__ t) {
  typedef typename ResidStore<S>::t RR;
  GROUP_LOOP(blas)
    k_ru_apply_body<RR, S>(r.rh, reinterpret_cast<RR*>(r.rl), reinterpret_cast<S*>(r.p), r.n, r.n,
                          r.st, bx, r.NB, 0, nullptr);
  }
}
#undef GROUP_LOOP

// ---- a new member's start (one member, its own grid) --------------------------
__global__ void __launch_bounds__(RT) m_dot_bb(const double* __restrict__ b, long n,
                                               double* __restrict__ part, int vec) {
  __shared__ double sh[RT];
  k_dot_body<double, double>(b, b, n, n, n, part, vec, blockIdx.x, gridDim.x, 0, sh);
}

__global__ void __launch_bounds__(RT) m_init(RhsState* st, const double* part, int NB,
                                             int max_iter) {
  __shared__ double sh[RT];
  k_init_state_body(st, part, NB, max_iter, 0, sh);
}

template <class S>
__global__ void __launch_bounds__(RT) m_zero(S* __restrict__ x, long n) {
  k_zero_body<S>(x, n, n, blockIdx.x, gridDim.x, 0, nullptr);
}

// ---- host side -------------------------------------------------------------------
bool words_ok(size_t elem, long n, std::initializer_list<const void*> ptrs) {
  if ((((size_t)n * elem) & 15) != 0) return false;
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) & 15) return false;
  return true;
}

// LDS of a grouped hop launch: the largest member's (cg: with the fused CG
// step's one double per thread)
size_t hop_lds_max(size_t real_bytes, size_t lstride, bool cg) {
  size_t m = 0;
  for (int Ls = kLsMin; Ls <= kLsMax; ++Ls) {
    const int nsb = 4 * (64 / Ls);
    m = std::max(m, (size_t)8 * lstride * nsb * real_bytes + (size_t)8 * nsb * sizeof(int) +
                        (cg ? 256 * sizeof(double) : 0));
  }
  return m;
}

size_t local_lds_max(size_t real_bytes) {
  size_t m = 0;
  for (int Ls = kLsMin; Ls <= kLsMax; ++Ls) m = std::max(m, local_lds_bytes(kLocalThreads, Ls, real_bytes));
  return m;
}

// The launches of one round: k x [reliable update; iteration].
template <class S, class R, int LAYOUT>
int record_round(const Table* t, int k, hipStream_t st) {
  typedef typename Store<S>::compute T;
  const size_t lds_s = hop_lds_max(sizeof(T), LinkStride<T>::v, true);
  const size_t lds_d = hop_lds_max(sizeof(double), LinkStride<double>::v, false);
  const size_t loc_s = local_lds_max(sizeof(T));
  const size_t loc_d = local_lds_max(sizeof(double));
  const dim3 hg(kHopGrid), hb(256), lg(kLocalGrid), lb(kLocalThreads), bg(kBlasGrid), bb(RT),
      og(kGroupMax);
  // M_pc (mid: between its two hops, for the fused CG step's reductions)
  // and M_pc^dag
  auto mpc = [&](auto stag, size_t lds, size_t llds, int fp64, int want) {
    typedef decltype(stag) P;
    // its first stage hands the second chi = (A/b) M_ee^-1 M_eo p
    hipLaunchKernelGGL((g_hop<P, LAYOUT, false, true, true, true>), hg, hb, lds, st, t, 0, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, false, false, false, false>), hg, hb, lds, st, t, 0, fp64, want);
    hipLaunchKernelGGL((g_local<P, LAYOUT>), lg, lb, llds, st, t, 0, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, false, true, false, true>), hg, hb, lds, st, t, 1, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, false, false, false, true>), hg, hb, lds, st, t, 1, fp64, want);
  };
  auto mpc_dag = [&](auto stag, size_t lds, size_t llds, int fp64, int want) {
    typedef decltype(stag) P;
    hipLaunchKernelGGL((g_hop<P, LAYOUT, true, true, true, false>), hg, hb, lds, st, t, 2, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, true, false, false, false>), hg, hb, lds, st, t, 2, fp64, want);
    hipLaunchKernelGGL((g_local<P, LAYOUT>), lg, lb, llds, st, t, 1, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, true, true, false, false>), hg, hb, lds, st, t, 3, fp64, want);
    hipLaunchKernelGGL((g_hop<P, LAYOUT, true, false, false, false>), hg, hb, lds, st, t, 3, fp64, want);
  };
  for (int i = 0; i < k; ++i) {
    // reliable update of the members that asked for one (and the initial one)
    hipLaunchKernelGGL((g_fold_x<R>), bg, bb, 0, st, t);
    mpc(double(), lds_d, loc_d, 1, ST_UPDATE);
    mpc_dag(double(), lds_d, loc_d, 1, ST_UPDATE);
    hipLaunchKernelGGL(g_resid, bg, bb, 0, st, t);
    hipLaunchKernelGGL(g_ru_decide, og, bb, 0, st, t);
    hipLaunchKernelGGL((g_ru_apply<S, R>), bg, bb, 0, st, t);
    // one iteration of the running members, its vector steps fused into
    // the last hops of M_pc and M_pc^dag
    mpc(S(), lds_s, loc_s, 0, ST_RUN);
    hipLaunchKernelGGL(g_sum_sites, bg, bb, 0, st, t);
    hipLaunchKernelGGL(g_alpha, og, bb, 0, st, t);
    mpc_dag(S(), lds_s, loc_s, 0, ST_RUN);
    hipLaunchKernelGGL(g_sum_sites, bg, bb, 0, st, t);
    hipLaunchKernelGGL(g_beta, og, bb, 0, st, t);
    hipLaunchKernelGGL((g_update_p<S>), bg, bb, 0, st, t);
  }
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

template <class F>
int by_types(int inner, int layout, F&& f) {
  auto lay = [&](auto stag, auto rtag) -> int {
    if (layout == QDWF_RIRI) return f(stag, rtag, std::integral_constant<int, QDWF_RIRI>());
    return f(stag, rtag, std::integral_constant<int, QDWF_RRII>());
  };
  switch (inner) {
    case QDWF_F64: return lay(double(), double());
    case QDWF_F32: return lay(float(), float());
    case QDWF_F16: return lay(_Float16(), float());
    case QDWF_BF16: return lay(bf16(), float());
  }
  return fail(QDWF_EINVAL, "unknown inner precision %d", inner);
}

int fill_hop(qdwf_ctx* ctx, int prec, const HopArgs& a, HopK* k) {
  const HopShape sh = {256, 1, 0, 0, 0};
  size_t lds = 0;
  int nb = 0;
  auto go = [&](auto stag) -> int {
    typedef decltype(stag) S;
    return a.minv ? make_hopk<S, true>(ctx, prec, a, sh, k, &lds, &nb)
                  : make_hopk<S, false>(ctx, prec, a, sh, k, &lds, &nb);
  };
  switch (prec) {
    case QDWF_F64: return go(double());
    case QDWF_F32: return go(float());
    case QDWF_F16: return go(_Float16());
    case QDWF_BF16: return go(bf16());
  }
  return fail(QDWF_EINVAL, "unknown precision %d", prec);
}

// Hop and local arguments of M_pc^dag M_pc (stages 0..3) on one member:
// out = M_pc^dag M_pc in with temporaries v, te1, te2 (half fields of prec).
// With cg (the inner iteration), the last hops of M_pc and M_pc^dag take the
// fused CG step instead (cg->mode is set per hop): out is then not written.
int fill_mdagm(qdwf_ctx* ctx, int prec, const void* in, void* out, void* v, void* te1, void* te2,
               HopK* hk[4], GLoc* lk[2], const CgFuse* cg = nullptr) {
  const Geom& g = ctx->g;
  const long rs = g.n5h * 24;
  const bool ls16 = g.Ls == 16;
  const double al = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
  const double be = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
  int rc;
  for (int dag = 0; dag < 2; ++dag) {
    const void* src = dag ? v : in;      // input of this M_pc (or M_pc^dag)
    void* dst = dag ? out : v;
    HopArgs a = {};
    a.in[QDWF_EVEN] = src;
    a.out[QDWF_EVEN] = ls16 ? te2 : te1;
    a.rs_in = a.rs_out = a.rs_z = rs;
    a.par0 = QDWF_EVEN;
    a.npar = 1;
    a.nrhs = 1;
    a.hop_scale = -0.5;
    a.minv = ls16 ? 1 : 0;
    a.chi = (ls16 && !dag) ? 1 : 0;
    if ((rc = fill_hop(ctx, prec, a, hk[2 * dag]))) return rc;
    GLoc& l = *lk[dag];
    l.in = te1;
    l.out = te2;
    const MatKind kind = dag ? MAT_MEEINV_DAG : MAT_AMEEINV;
    const size_t off = (size_t)kind * 2 * g.Ls * g.Ls;
    l.K = prec == QDWF_F64 ? (const void*)(ctx->d_mat64 + off) : (const void*)(ctx->d_mat32 + off);
    l.Vh = g.Vh;
    l.Ls = g.Ls;
    l.plane = g.n5h;
    HopArgs b = {};
    b.in[QDWF_ODD] = te2;
    b.out[QDWF_ODD] = dst;
    b.z[QDWF_ODD] = src;
    b.rs_in = b.rs_out = b.rs_z = rs;
    b.par0 = QDWF_ODD;
    b.npar = 1;
    b.nrhs = 1;
    b.epi = 1;
    b.hop_scale = 0.5;
    b.alpha = al;
    b.beta = be;
    b.chi = dag ? 0 : 1;
    if (cg) {
      b.cg = dag ? (cg->x ? 3 : 2) : 1;
      b.cg_r = cg->r;
      b.cg_alpha = cg->alpha;
      b.cg_alpha_stride = cg->alpha_stride;
      b.cg_site = cg->site;
      b.cg_x = cg->x;
      b.cg_p = cg->p;
    }
    if ((rc = fill_hop(ctx, prec, b, hk[2 * dag + 1]))) return rc;
  }
  return QDWF_OK;
}

}  // namespace

size_t group_table_bytes() { return al256(sizeof(Table)); }

int GroupEngine::create(int device, int inner, int layout, int k, void* table_mem,
                        hipStream_t capture, GroupEngine** out) {
  *out = nullptr;
  if (k < 1 || k > 64) return fail(QDWF_EINVAL, "iterations per round %d out of [1, 64]", k);
  if (!capture) return fail(QDWF_EINVAL, "a capture stream is needed");
  GroupEngine* e = new (std::nothrow) GroupEngine();
  if (!e) return fail(QDWF_ENOMEM, "host allocation failed");
  e->device_ = device;
  e->inner_ = inner;
  e->layout_ = layout;
  e->k_ = k;
  e->table_ = table_mem;
  if (hipHostMalloc(&e->staging_, sizeof(Table)) != hipSuccess) {
    e->staging_ = nullptr;
    delete e;
    return fail(QDWF_ENOMEM, "pinned host staging of %zu bytes failed", sizeof(Table));
  }
  std::memset(e->staging_, 0, sizeof(Table));
  int rc = e->capture(capture);
  if (rc) {
    delete e;
    return rc;
  }
  *out = e;
  return QDWF_OK;
}

int GroupEngine::capture(hipStream_t cs) {
  QDWF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const Table* t = reinterpret_cast<const Table*>(table_);
  int rc = by_types(inner_, layout_, [&](auto stag, auto rtag, auto lay) -> int {
    return record_round<decltype(stag), decltype(rtag), decltype(lay)::value>(t, k_, cs);
  });
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(QDWF_EDEVICE, "capture of the round failed: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&exec_, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    exec_ = nullptr;
    return fail(QDWF_EDEVICE, "instantiation of the round failed: %s", hipGetErrorString(e2));
  }
  return QDWF_OK;
}

GroupEngine::~GroupEngine() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (staging_) (void)hipHostFree(staging_);
}

int GroupEngine::set_members(const GroupMember* m, int n, hipStream_t st) {
  if (n < 0 || n > kGroupMax) return fail(QDWF_EINVAL, "%d members, at most %d", n, kGroupMax);
  Table& T = *reinterpret_cast<Table*>(staging_);
  T.blas.n = T.one.n = T.hop16.n = T.hopg.n = T.loc.n = T.sites.n = n;
  T.blas.start[0] = T.one.start[0] = T.hop16.start[0] = T.hopg.start[0] = T.loc.start[0] =
      T.sites.start[0] = 0;
  const size_t ps = prec_bytes(inner_);
  const size_t rsz = inner_ == QDWF_F64 ? 8 : 4;
  int rc;
  for (int j = 0; j < n; ++j) {
    qdwf_ctx* c = m[j].ctx;
    const Geom& g = c->g;
    if (g.Ls < kLsMin || g.Ls > kLsMax)
      return fail(QDWF_EINVAL, "grouped solves take %d <= Ls <= %d (got %d)", kLsMin, kLsMax, g.Ls);
    const long n5 = g.n5h * 24;
    const Layout L = solver_layout(n5, 1, inner_);
    char* w = m[j].ws;
    GReq& r = T.req[j];
    r.st = m[j].st;
    r.n = n5;
    r.NB = reduce_blocks(n5);
    r.nsite = g.Vh;
    r.NBs = site_blocks(g.Vh);
    // the per-site sums take the room of Ap, which the fused iteration never stores
    r.site = reinterpret_cast<double*>(w + L.off_ap);
    r.xl = w + L.off_xl;
    r.rl = w + L.off_rl;
    r.p = w + L.off_p;
    r.ap = w + L.off_ap;
    r.xh = m[j].xo;
    r.b = m[j].bo;
    r.rh = reinterpret_cast<double*>(w + L.off_rh);
    r.ax = reinterpret_cast<double*>(w + L.off_ax);
    r.part = reinterpret_cast<double*>(w + L.off_part);
    r.vec_s = words_ok(ps, n5, {r.p}) ? 1 : 0;
    r.vec_r = words_ok(rsz, n5, {r.xl}) && words_ok(inner_ == QDWF_F16 ? 2 : rsz, n5, {r.rl}) ? 1 : 0;
    r.vec_b = words_ok(8, n5, {r.b}) ? 1 : 0;
    r.scale = inner_ != QDWF_F64 ? 1 : 0;
    r.max_iter = m[j].max_iter > 0 ? m[j].max_iter : 20000;
    r.tol2 = m[j].tol * m[j].tol;
    const double delta = m[j].delta > 0 ? m[j].delta : 0.1;
    r.delta2 = inner_ == QDWF_F64 ? 0.0 : delta * delta;
    HopK* hs[4] = {&T.hop_s[0][j], &T.hop_s[1][j], &T.hop_s[2][j], &T.hop_s[3][j]};
    GLoc* ls[2] = {&T.loc_s[0][j], &T.loc_s[1][j]};
    const double* alpha = reinterpret_cast<const double*>(reinterpret_cast<const char*>(r.st) +
                                                          offsetof(RhsState, alpha));
    const CgFuse cg = {0, r.rl, alpha, 0, r.site, r.xl, r.p};
    if ((rc = fill_mdagm(c, inner_, r.p, r.ap, w + L.off_v, w + L.off_t1, w + L.off_t2, hs, ls, &cg)))
      return rc;
    HopK* hd[4] = {&T.hop_d[0][j], &T.hop_d[1][j], &T.hop_d[2][j], &T.hop_d[3][j]};
    GLoc* ld[2] = {&T.loc_d[0][j], &T.loc_d[1][j]};
    if ((rc = fill_mdagm(c, QDWF_F64, r.xh, r.ax, w + L.off_vh, w + L.off_t1h, w + L.off_t2h, hd, ld)))
      return rc;
    const int gpw = 64 / g.Ls;
    T.blas.start[j + 1] = T.blas.start[j] + r.NB;
    T.sites.start[j + 1] = T.sites.start[j] + r.NBs;
    T.one.start[j + 1] = j + 1;
    const int hop_units = (g.Vh + 4 * gpw - 1) / (4 * gpw);
    T.hop16.start[j + 1] = T.hop16.start[j] + (g.Ls == 16 ? hop_units : 0);
    T.hopg.start[j + 1] = T.hopg.start[j] + (g.Ls == 16 ? 0 : hop_units);
    const int G = (kLocalThreads / 64) * gpw;
    T.loc.start[j + 1] = T.loc.start[j] + (g.Ls == 16 ? 0 : (g.Vh + G - 1) / G);
  }
  QDWF_HIP(hipMemcpyAsync(table_, staging_, sizeof(Table), hipMemcpyHostToDevice, st));
  return QDWF_OK;
}

int GroupEngine::start_member(const GroupMember& m, hipStream_t st) {
  const long n5 = m.ctx->g.n5h * 24;
  const int NB = reduce_blocks(n5);
  const Layout L = solver_layout(n5, 1, inner_);
  double* part = reinterpret_cast<double*>(m.ws + L.off_part);
  hipLaunchKernelGGL(m_dot_bb, dim3(NB), dim3(RT), 0, st, m.bo, n5, part,
                     words_ok(8, n5, {m.bo}) ? 1 : 0);
  hipLaunchKernelGGL(m_init, dim3(1), dim3(RT), 0, st, m.st, part, NB,
                     m.max_iter > 0 ? m.max_iter : 20000);
  if (inner_ == QDWF_F64)
    hipLaunchKernelGGL((m_zero<double>), dim3(NB), dim3(RT), 0, st,
                       reinterpret_cast<double*>(m.ws + L.off_xl), n5);
  else
    hipLaunchKernelGGL((m_zero<float>), dim3(NB), dim3(RT), 0, st,
                       reinterpret_cast<float*>(m.ws + L.off_xl), n5);
  hipLaunchKernelGGL((m_zero<double>), dim3(NB), dim3(RT), 0, st, m.xo, n5);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

int GroupEngine::launch_round(hipStream_t st) {
  QDWF_HIP(hipGraphLaunch(exec_, st));
  return QDWF_OK;
}

}  // namespace qdwf
