// Conjugate gradient on the even-odd preconditioned normal operator
// M_pc^dag M_pc, for several right-hand sides at once, with
//   * plain FP64 CG (inner precision FP64), or
//   * reliable-update mixed-precision CG: the inner iteration runs its Dslash
//     on FP32 arithmetic with FP32, FP16 or BF16 storage of p and the
//     operator temporaries, r in FP32 (in FP16 with FP16 storage) and the
//     solution increment in FP32, all dot
//     products accumulated in FP64; when the inner residual has dropped by
//     delta since the last update (or reached the target) the increment is
//     folded into the FP64 solution and the residual is recomputed in FP64
//     from b - A x (Sleijpen and van der Vorst's reliable updates). The solve
//     ends only on the FP64 true residual.
// The inner vectors are kept scaled to unit RMS (scale sigma per rhs, reset at
// each reliable update), which keeps FP16 storage clear of its subnormal range.
//
// Every per-iteration scalar (alpha, beta, |r|^2, status) lives on the device
// in a RhsState per right-hand side, so an iteration is a fixed sequence of
// launches with no host round trip; it can be captured once in a HIP graph and
// replayed. Reductions are two-stage with a block count that depends only on
// the field size and a fixed summation tree, so each right-hand side's result
// is bitwise independent of what else is in the batch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <initializer_list>

#include <cstddef>

#include "cgbody.h"

namespace qdwf {

namespace {

// Launches over one context's right-hand sides: grid x = blocks of a field,
// y = right-hand side (per-right-hand-side steps: x = right-hand side).
template <class SA, class SB>
__global__ void __launch_bounds__(RT) k_dot(const SA* __restrict__ a, const SB* __restrict__ b,
                                            long n, long rsa, long rsb, double* __restrict__ part,
                                            int vec) {
  __shared__ double sh[RT];
  k_dot_body<SA, SB>(a, b, n, rsa, rsb, part, vec, blockIdx.x, gridDim.x, blockIdx.y, sh);
}

__global__ void __launch_bounds__(RT) k_alpha(const double* __restrict__ part, int NB,
                                              RhsState* __restrict__ st, int j) {
  __shared__ double sh[RT];
  k_alpha_body(part, NB, st, blockIdx.x, sh, j);
}

__global__ void __launch_bounds__(RT) k_beta(const double* __restrict__ part, int NB,
                                             RhsState* __restrict__ st, double delta2, int j) {
  __shared__ double sh[RT];
  k_beta_body(part, NB, st, delta2, blockIdx.x, sh, j);
}

template <class SR, class SP>
__global__ void __launch_bounds__(RT) k_grp_p(const SR* __restrict__ r, SP* __restrict__ p0, long ps,
                                              int j, long n, const RhsState* __restrict__ st,
                                              int vec) {
  k_grp_p_body<SR, SP>(r, p0, ps, j, n, n, st, vec, blockIdx.x, gridDim.x, blockIdx.y);
}

template <class SX, class SR, class SP>
__global__ void __launch_bounds__(RT) k_grp_last(SX* __restrict__ x, const SR* __restrict__ r,
                                                 SP* __restrict__ p0, long ps, int len, long n,
                                                 const RhsState* __restrict__ st, int vec) {
  k_grp_last_body<SX, SR, SP>(x, r, p0, ps, len, n, n, st, vec, blockIdx.x, gridDim.x, blockIdx.y);
}

__global__ void __launch_bounds__(RT) k_sum_sites(const double* __restrict__ v, long n,
                                                  double* __restrict__ part) {
  __shared__ double sh[RT];
  k_sum_body(v, n, part, blockIdx.x, gridDim.x, blockIdx.y, sh);
}

template <class SX>
__global__ void __launch_bounds__(RT) k_fold_x(double* __restrict__ xh, SX* __restrict__ xl,
                                               long n, long rs_h, long rs,
                                               const RhsState* __restrict__ st) {
  k_fold_x_body<SX>(xh, xl, n, rs_h, rs, st, blockIdx.x, gridDim.x, blockIdx.y, nullptr);
}

__global__ void __launch_bounds__(RT) k_resid(const double* __restrict__ b,
                                              const double* __restrict__ Ax,
                                              double* __restrict__ rh, long n, long rs_b,
                                              long rs, double* __restrict__ part) {
  __shared__ double sh[RT];
  k_resid_body(b, Ax, rh, n, rs_b, rs, part, blockIdx.x, gridDim.x, blockIdx.y, sh);
}

__global__ void __launch_bounds__(RT) k_ru_decide(const double* __restrict__ part, int NB,
                                                  RhsState* __restrict__ st, double tol2,
                                                  double nreal, int scale, int first) {
  __shared__ double sh[RT];
  k_ru_decide_body(part, NB, st, tol2, nreal, scale, first, blockIdx.x, sh);
}

template <class SR, class SP>
__global__ void __launch_bounds__(RT) k_ru_apply(const double* __restrict__ rh,
                                                 SR* __restrict__ rl, SP* __restrict__ p, long n,
                                                 long rs, const RhsState* __restrict__ st) {
  k_ru_apply_body<SR, SP>(rh, rl, p, n, rs, st, blockIdx.x, gridDim.x, blockIdx.y, nullptr);
}

__global__ void k_init_state(RhsState* st, const double* part, int NB) {
  __shared__ double sh[RT];
  k_init_state_body(st, part, NB, 0, blockIdx.x, sh);
}

template <class S>
__global__ void k_zero(S* __restrict__ x, long n, long rs) {
  k_zero_body<S>(x, n, rs, blockIdx.x, gridDim.x, blockIdx.y, nullptr);
}

// Imaginary part of <a, b> = sum a_re b_im - a_im b_re, per layout.
template <class SA, class SB, int LAYOUT>
__global__ void __launch_bounds__(RT) k_dot_im(const SA* __restrict__ a, const SB* __restrict__ b,
                                               long n, long rsa, long rsb, long plane,
                                               double* __restrict__ part) {
  __shared__ double sh[RT];
  const int r = blockIdx.y, NB = gridDim.x;
  const SA* ar = a + (long)r * rsa;
  const SB* br = b + (long)r * rsb;
  double acc = 0;
  const long nc = n / 2;   // complex numbers
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < nc; i += (long)NB * RT) {
    long ire, iim;
    if (LAYOUT == QDWF_RIRI) {
      ire = 2 * i;
      iim = 2 * i + 1;
    } else {
      // half fields of 24*plane reals: [re planes 0..11][im planes 0..11]
      const long h = i / (12 * plane), w = i - h * 12 * plane;
      ire = h * 24 * plane + w;
      iim = ire + 12 * plane;
    }
    acc += rd(ar, ire) * rd(br, iim) - rd(ar, iim) * rd(br, ire);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)r * NB + blockIdx.x] = t;
}

__global__ void __launch_bounds__(RT) k_sum(const double* __restrict__ part, int NB,
                                            double* __restrict__ out, int stride) {
  __shared__ double sh[RT];
  const int r = blockIdx.x;
  double acc = 0;
  for (int i = threadIdx.x; i < NB; i += RT) acc += part[(long)r * NB + i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[(long)r * stride] = t;
}

__global__ void k_force_update(RhsState* st, int nrhs) {
  for (int q = threadIdx.x; q < nrhs; q += blockDim.x)
    if (st[q].status == ST_RUN) st[q].status = ST_UPDATE;
}

template <class S>
__global__ void k_copy64(double* __restrict__ d, const S* __restrict__ s, long n, long rs_d,
                         long rs_s) {
  const int q = blockIdx.y, NB = gridDim.x;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)NB * RT)
    d[(long)q * rs_d + i] = (double)Store<S>::to(s[(long)q * rs_s + i]);
}

}  // namespace

// Blocks of the reduction of per-site sums (a few values per thread: the
// sums are few and the reduction sits between two hops of an iteration).
// Never more than reduce_blocks gives for the 2 x 24 x Ls x sites reals of
// the same field, whose partials share the room.
int site_blocks(long nsite) {
  long nb = (nsite + 1023) / 1024;
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;
  return (int)nb;
}

int reduce_blocks(long n) {
  long nb = (n + 8191) / 8192;
  if (nb < 1) nb = 1;
  if (nb > 2048) nb = 2048;   // 8 blocks per CU at most; the second stage sums them in one block
  return (int)nb;
}

// ---- operator compositions ---------------------------------------------------
int apply_hop_parity(qdwf_ctx* ctx, int prec, int layout, int dagger, int out_par, void* out,
                     const void* in, const void* z, double scale, int nrhs, long rs,
                     hipStream_t st, const int* skip, int skip_stride) {
  HopArgs a = {};
  a.skip = skip;
  a.skip_stride = skip_stride;
  a.in[out_par] = in;
  a.out[out_par] = out;
  a.z[out_par] = z;
  a.rs_in = a.rs_out = a.rs_z = rs;
  a.par0 = out_par;
  a.npar = 1;
  a.nrhs = nrhs;
  a.epi = z != nullptr;
  a.hop_scale = scale;
  const double al = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
  const double be = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
  a.alpha = al;
  a.beta = be;
  return launch_hop(ctx, prec, layout, dagger, a, st);
}

// out = M_pc in (dagger 0) or M_pc^dag in; te1, te2: even half fields.
// For M_pc the first stage leaves chi = (A/b) M_ee^-1 M_eo in in te2 (A/b
// and M_ee^-1 commute, both being functions of C), so the second hop takes
// its input as it is instead of applying A to each of its 8 neighbours;
// M_pc^dag applies A^dag once per site inside its hops anyway.
int apply_mpc(qdwf_ctx* ctx, int prec, int layout, int dagger, void* out, const void* in,
              void* te1, void* te2, int nrhs, long rs, hipStream_t st, const int* skip,
              int skip_stride, const CgFuse* cg) {
  int rc;
  const int chi = dagger ? 0 : 1;
  if (ctx->g.Ls == 16) {
    // te2 = M_ee^-1 M_eo in (times A/b), or M_ee^-dag (M_oe)^dag in, in one
    // launch: the hop's 16 slices of a site share a DPP row, where M_ee^-1 is
    // a scan
    HopArgs a = {};
    a.in[QDWF_EVEN] = in;
    a.out[QDWF_EVEN] = te2;
    a.rs_in = a.rs_out = a.rs_z = rs;
    a.par0 = QDWF_EVEN;
    a.npar = 1;
    a.nrhs = nrhs;
    a.hop_scale = -0.5;
    a.minv = 1;
    a.chi = chi;
    a.skip = skip;
    a.skip_stride = skip_stride;
    if ((rc = launch_hop(ctx, prec, layout, dagger, a, st))) return rc;
  } else {
    // te1 = M_eo in  (or (M_oe)^dag in), then te2 = (A/b) M_ee^-1 te1 (or M_ee^-dag te1)
    if ((rc = apply_hop_parity(ctx, prec, layout, dagger, QDWF_EVEN, te1, in, nullptr, -0.5, nrhs,
                               rs, st, skip, skip_stride)))
      return rc;
    if ((rc = launch_local(ctx, prec, layout, dagger ? MAT_MEEINV_DAG : MAT_AMEEINV, te2, te1, 1, 0,
                           rs, nrhs, st)))
      return rc;
  }
  // out = M_oo in - M_oe te2 = alpha in + beta C in + 1/2 D_h A te2
  // (for M_pc the hop takes chi = A te2 / b from te2)
  HopArgs a = {};
  a.in[QDWF_ODD] = te2;
  a.out[QDWF_ODD] = out;
  a.z[QDWF_ODD] = in;
  a.rs_in = a.rs_out = a.rs_z = rs;
  a.par0 = QDWF_ODD;
  a.npar = 1;
  a.nrhs = nrhs;
  a.epi = 1;
  a.hop_scale = 0.5;
  a.alpha = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
  a.beta = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
  a.chi = chi;
  a.skip = skip;
  a.skip_stride = skip_stride;
  if (cg) {
    a.cg = cg->mode;
    a.cg_r = cg->r;
    a.cg_alpha = cg->alpha;
    a.cg_alpha_stride = cg->alpha_stride;
    a.cg_site = cg->site;
    a.cg_x = cg->x;
    a.cg_p = cg->p;
  }
  return launch_hop(ctx, prec, layout, dagger, a, st);
}

int apply_mdagm(qdwf_ctx* ctx, int prec, int layout, void* out, const void* in, void* v,
                void* te1, void* te2, int nrhs, long rs, hipStream_t st, const int* skip,
                int skip_stride) {
  int rc;
  if ((rc = apply_mpc(ctx, prec, layout, 0, v, in, te1, te2, nrhs, rs, st, skip, skip_stride)))
    return rc;
  return apply_mpc(ctx, prec, layout, 1, out, v, te1, te2, nrhs, rs, st, skip, skip_stride);
}

int dot_re_im(qdwf_ctx* ctx, double* out_host, const void* x, const void* y, long n, int prec,
              int layout, int nrhs, void* ws, hipStream_t st) {
  const int NB = reduce_blocks(n);
  double* part = reinterpret_cast<double*>(ws);
  double* res = part + (long)NB * nrhs;
  auto go = [&](auto tag) -> int {
    typedef decltype(tag) S;
    const S* a = reinterpret_cast<const S*>(x);
    const S* b = reinterpret_cast<const S*>(y);
    const int vec = vec_ok<S>(n, {a, b}) ? 1 : 0;
    hipLaunchKernelGGL((k_dot<S, S>), dim3(NB, nrhs), dim3(RT), 0, st, a, b, n, n, n, part, vec);
    hipLaunchKernelGGL(k_sum, dim3(nrhs), dim3(RT), 0, st, part, NB, res, 2);
    if (layout == QDWF_RIRI)
      hipLaunchKernelGGL((k_dot_im<S, S, QDWF_RIRI>), dim3(NB, nrhs), dim3(RT), 0, st, a, b, n, n, n,
                         ctx->g.n5h, part);
    else
      hipLaunchKernelGGL((k_dot_im<S, S, QDWF_RRII>), dim3(NB, nrhs), dim3(RT), 0, st, a, b, n, n, n,
                         ctx->g.n5h, part);
    hipLaunchKernelGGL(k_sum, dim3(nrhs), dim3(RT), 0, st, part, NB, res + 1, 2);
    QDWF_HIP(hipGetLastError());
    QDWF_HIP(hipMemcpyAsync(out_host, res, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, st));
    QDWF_HIP(hipStreamSynchronize(st));
    return QDWF_OK;
  };
  switch (prec) {
    case QDWF_F64: return go(double());
    case QDWF_F32: return go(float());
    case QDWF_F16: return go(_Float16());
    case QDWF_BF16: return go(bf16());
  }
  return fail(QDWF_EINVAL, "unknown precision %d", prec);
}

void forget_graph(qdwf_ctx* c) {
  if (c->graph.exec) (void)hipGraphExecDestroy(c->graph.exec);
  c->graph = SolveGraph();
}

void forget_solver_state(qdwf_ctx* c) {
  forget_graph(c);
  if (c->ev) (void)hipEventDestroy(c->ev);
  c->ev = nullptr;
  if (c->h_pin) (void)hipHostFree(c->h_pin);
  c->h_pin = nullptr;
  c->h_pin_bytes = 0;
}

size_t dot_ws_bytes(long n, int nrhs) {
  return sizeof(double) * ((size_t)reduce_blocks(n) * nrhs + 2 * (size_t)nrhs) + 256;
}

// ---- the solver ----------------------------------------------------------------

Layout solver_layout(long n, int nrhs, int inner, bool grouped) {
  Layout L;
  const size_t sS = prec_bytes(inner);
  const size_t sR = inner == QDWF_F64 ? 8 : 4;
  const size_t sRl = inner == QDWF_F16 ? 2 : sR;   // the residual's storage (ResidStore)
  const size_t v64 = al256(8 * (size_t)n * nrhs);
  const size_t vR = al256(sR * (size_t)n * nrhs);
  const size_t vS = al256(sS * (size_t)n * nrhs);
  size_t o = 0;
  L.off_rh = o; o += v64;
  L.off_ax = o; o += v64;
  L.off_vh = o; o += v64;
  L.off_t1h = o; o += v64;
  L.off_t2h = o; o += v64;
  L.off_xl = o; o += vR;
  L.off_rl = o; o += al256(sRl * (size_t)n * nrhs);
  L.off_p = o; o += vS * (grouped ? kGroupSlots : 1);
  L.off_ap = o; o += vS;
  L.off_v = o; o += vS;
  L.off_t1 = o; o += vS;
  L.off_t2 = o; o += vS;
  // partials: room for one reduction over 2n reals per rhs plus 2 results per rhs
  L.off_part = o; o += al256(sizeof(double) * ((size_t)reduce_blocks(2 * n) * nrhs + 2 * (size_t)nrhs));
  L.off_state = o; o += al256(sizeof(RhsState) * (size_t)nrhs);
  L.off_stage = o; o += al256(8 * (size_t)n * nrhs * 2);   // FULL: source prep / rhs
  L.total = o;
  return L;
}

namespace {

template <class S, class R>
struct Cg {
  typedef typename ResidStore<S>::t RR;   // storage of the inner residual
  qdwf_ctx* ctx;
  hipStream_t st;
  int layout, inner, nrhs;
  long n;            // reals per rhs (half field)
  int NB;
  char* ws;
  Layout L;
  double* xh;        // FP64 solution (odd half fields), stride rs_x
  long rs_x;
  const double* b;   // FP64 right-hand side (odd half fields), stride rs_b
  long rs_b;
  RhsState* d_state;
  std::vector<RhsState> h_state;
  double delta2, tol2;
  int64_t hop_applications;

  template <class X> X* at(size_t off) { return reinterpret_cast<X*>(ws + off); }
  double* part() { return at<double>(L.off_part); }
  dim3 grid() const { return dim3(NB, nrhs); }

  // One CG iteration with its vector work fused into the operator's hops:
  //   v = M_pc p, with |v|^2 = <p, M_pc^dag M_pc p> summed by the hop;
  //   alpha = |r|^2 / |v|^2;
  //   r -= alpha M_pc^dag v inside the last hop (Ap is never stored), with
  //   |r|^2 summed there;
  //   beta; p = r + beta p, and x += alpha p once per group of iterations.
  // The hops leave one sum per checkerboard site (in the room of Ap), which
  // k_sum_sites reduces with a block count that depends only on the field size.
  // Iterations come in groups of up to kGroupSlots (iteration j of a group
  // of len): iteration j reads p from slot j and writes the next p to slot
  // j + 1; the last one adds every step of the group to x in one pass and
  // writes the next p to slot 0, where every group starts.
  int inner_iteration(int j, int len) {
    int rc;
    S* p0 = at<S>(L.off_p);
    const long ps = (long)(al256(prec_bytes(inner) * (size_t)n * nrhs) / prec_bytes(inner));
    S* p = p0 + (long)j * ps;
    S* v = at<S>(L.off_v);
    R* x = at<R>(L.off_xl);
    RR* r = at<RR>(L.off_rl);
    double* site = at<double>(L.off_ap);
    const long nsite = ctx->g.Vh;
    const int NBs = site_blocks(nsite);
    // the workspace arrays start on 256-byte boundaries and n is a multiple of 24
    const int vec = vec_ok<S>(n, {p0}) && vec_ok<R>(n, {x}) && vec_ok<RR>(n, {r}) ? 1 : 0;
    // the hops of a right-hand side that is not running do no work
    static_assert(sizeof(RhsState) % sizeof(double) == 0, "RhsState is read as ints and doubles");
    const int* skip = reinterpret_cast<const int*>(
        reinterpret_cast<const char*>(d_state) + offsetof(RhsState, status));
    const int sk = (int)(sizeof(RhsState) / sizeof(int));
    CgFuse f1 = {1, nullptr, nullptr, 0, site};
    if ((rc = apply_mpc(ctx, inner, layout, 0, v, p, at<S>(L.off_t1), at<S>(L.off_t2), nrhs, n, st,
                        skip, sk, &f1)))
      return rc;
    hipLaunchKernelGGL(k_sum_sites, dim3(NBs, nrhs), dim3(RT), 0, st, site, nsite, part());
    hipLaunchKernelGGL(k_alpha, dim3(nrhs), dim3(RT), 0, st, part(), NBs, d_state, j);
    const double* alpha = reinterpret_cast<const double*>(
        reinterpret_cast<const char*>(d_state) + offsetof(RhsState, alpha));
    CgFuse f2 = {2, r, alpha, (int)(sizeof(RhsState) / sizeof(double)), site};
    if ((rc = apply_mpc(ctx, inner, layout, 1, at<S>(L.off_ap), v, at<S>(L.off_t1), at<S>(L.off_t2),
                        nrhs, n, st, skip, sk, &f2)))
      return rc;
    hipLaunchKernelGGL(k_sum_sites, dim3(NBs, nrhs), dim3(RT), 0, st, site, nsite, part());
    hipLaunchKernelGGL(k_beta, dim3(nrhs), dim3(RT), 0, st, part(), NBs, d_state, delta2, j);
    if (j + 1 < len)
      hipLaunchKernelGGL((k_grp_p<RR, S>), grid(), dim3(RT), 0, st, r, p0, ps, j, n, d_state, vec);
    else
      hipLaunchKernelGGL((k_grp_last<R, RR, S>), grid(), dim3(RT), 0, st, x, r, p0, ps, len, n,
                         d_state, vec);
    QDWF_HIP(hipGetLastError());
    hop_applications += 4;
    return QDWF_OK;
  }

  // count iterations in groups of up to kGroupSlots: after them x holds
  // every step and the next direction is in slot 0
  int inner_run(int count) {
    int rc = 0;
    for (int g = 0; g < count && !rc; g += kGroupSlots) {
      const int len = std::min(kGroupSlots, count - g);
      for (int j = 0; j < len && !rc; ++j) rc = inner_iteration(j, len);
    }
    return rc;
  }

  // FP64 true residual and restart of the inner recursion (first: initial setup)
  int reliable_update(bool first) {
    int rc;
    double* rh = at<double>(L.off_rh);
    double* ax = at<double>(L.off_ax);
    if (!first)
      hipLaunchKernelGGL((k_fold_x<R>), grid(), dim3(RT), 0, st, xh, at<R>(L.off_xl), n, rs_x, n,
                         d_state);
    if ((rc = apply_mdagm(ctx, QDWF_F64, layout, ax, xh, at<double>(L.off_vh),
                          at<double>(L.off_t1h), at<double>(L.off_t2h), nrhs, rs_x, st)))
      return rc;
    hop_applications += 4;
    hipLaunchKernelGGL(k_resid, grid(), dim3(RT), 0, st, b, ax, rh, n, rs_b, n, part());
    hipLaunchKernelGGL(k_ru_decide, dim3(nrhs), dim3(RT), 0, st, part(), NB, d_state, tol2,
                       (double)n, inner != QDWF_F64 ? 1 : 0, first ? 1 : 0);
    hipLaunchKernelGGL((k_ru_apply<RR, S>), grid(), dim3(RT), 0, st, rh, at<RR>(L.off_rl),
                       at<S>(L.off_p), n, n, d_state);
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
  }

  // ---- resumable driver: begin(), then alternately complete() and launch()
  qdwf_solve_params prm;
  RhsState* h_pin = nullptr;     // pinned host copy of the device states (the context's)
  hipEvent_t ev = nullptr;       // the context's round event
  int status = QDWF_OK;
  bool final_round = false;

  ~Cg() {
  }

  int fetch_async() {
    QDWF_HIP(hipMemcpyAsync(h_pin, d_state, sizeof(RhsState) * nrhs, hipMemcpyDeviceToHost, st));
    QDWF_HIP(hipEventRecord(ev, st));
    return QDWF_OK;
  }

  int begin() {
    int rc;
    d_state = at<RhsState>(L.off_state);
    hop_applications = 0;
    // the pinned state copy and the event belong to the context and are
    // reused by its later solves (the copy grows only for more rhs)
    const size_t need = sizeof(RhsState) * nrhs;
    if (ctx->h_pin_bytes < need) {
      if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
      ctx->h_pin = nullptr;
      ctx->h_pin_bytes = 0;
      QDWF_HIP(hipHostMalloc(&ctx->h_pin, need));
      ctx->h_pin_bytes = need;
    }
    if (!ctx->ev) QDWF_HIP(hipEventCreateWithFlags(&ctx->ev, hipEventDisableTiming));
    h_pin = reinterpret_cast<RhsState*>(ctx->h_pin);
    ev = ctx->ev;
    hipLaunchKernelGGL((k_dot<double, double>), grid(), dim3(RT), 0, st, b, b, n, rs_b, rs_b, part(),
                       vec_ok<double>(rs_b, {b}) ? 1 : 0);
    hipLaunchKernelGGL(k_init_state, dim3(nrhs), dim3(RT), 0, st, d_state, part(), NB);
    hipLaunchKernelGGL((k_zero<R>), grid(), dim3(RT), 0, st, at<R>(L.off_xl), n, n);
    if (!prm.x0_is_guess) hipLaunchKernelGGL((k_zero<double>), grid(), dim3(RT), 0, st, xh, n, rs_x);
    QDWF_HIP(hipGetLastError());
    if ((rc = reliable_update(true))) return rc;
    return fetch_async();
  }

  // Waits for the last launched round and decides; *finished is set once the
  // solve is over (status holds the outcome).
  int complete(bool* finished) {
    QDWF_HIP(hipEventSynchronize(ev));
    h_state.assign(h_pin, h_pin + nrhs);
    bool any_run = false, any_upd = false, bad = false;
    for (const RhsState& s : h_state) {
      any_run |= s.status == ST_RUN;
      any_upd |= s.status == ST_UPDATE;
      bad |= s.status == ST_NAN || s.status == ST_BREAKDOWN;
    }
    *finished = false;
    if (bad) { status = QDWF_ENAN; *finished = true; }
    else if (final_round) {
      bool all_done = true;
      for (const RhsState& s : h_state) all_done &= s.status == ST_DONE;
      status = all_done ? QDWF_OK : QDWF_ENOTCONV;
      *finished = true;
    } else if (!any_run && !any_upd) { status = QDWF_OK; *finished = true; }
    return QDWF_OK;
  }

  // Launches the next round (asynchronously): a reliable update if one is
  // due, otherwise `check_every` inner iterations; ends with a state fetch.
  int launch() {
    int rc = 0;
    bool any_upd = false;
    int max_it = 0;
    for (const RhsState& s : h_state) {
      any_upd |= s.status == ST_UPDATE;
      if (s.status == ST_RUN && s.iters > max_it) max_it = s.iters;
    }
    const int k = prm.check_every > 0 ? prm.check_every : 8;
    const int max_iter = prm.max_iter > 0 ? prm.max_iter : 20000;
    if (any_upd) {
      if ((rc = reliable_update(false))) return rc;
      return fetch_async();
    }
    if (max_it >= max_iter) {
      // out of iterations: fold the pending increment into x and report the
      // true residual of what the solve reached
      hipLaunchKernelGGL(k_force_update, dim3(1), dim3(64), 0, st, d_state, nrhs);
      if ((rc = reliable_update(false))) return rc;
      final_round = true;
      return fetch_async();
    }
    const int batch = std::min(k, max_iter - max_it);
    if (prm.use_graph && batch == k) {
      // the k iterations touch only the workspace, so one captured graph
      // serves every later solve of this context with the same workspace,
      // right-hand-side count, precisions, k and delta
      SolveGraph& G = ctx->graph;
      if (!(G.exec && G.ws == ws && G.nrhs == nrhs && G.inner == inner && G.layout == layout &&
            G.k == k && G.delta2 == delta2)) {
        forget_graph(ctx);
        QDWF_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int64_t h0 = hop_applications;
        rc = inner_run(k);
        hop_applications = h0;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc) {
          if (graph) (void)hipGraphDestroy(graph);
          return rc;
        }
        if (e != hipSuccess) return fail(QDWF_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        hipGraphExec_t exec = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess)
          return fail(QDWF_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e2));
        G.exec = exec;
        G.ws = ws;
        G.nrhs = nrhs;
        G.inner = inner;
        G.layout = layout;
        G.k = k;
        G.delta2 = delta2;
      }
      QDWF_HIP(hipGraphLaunch(G.exec, st));
      hop_applications += 4 * k;
    } else {
      rc = 0;
      rc = inner_run(batch);
      if (rc) return rc;
    }
    return fetch_async();
  }

  int result() const { return status; }

  void fill_stats(qdwf_solve_stats* stats) const {
    if (!stats) return;
    stats->iterations = 0;
    stats->reliable_updates = 0;
    stats->converged = 0;
    stats->true_residual = 0;
    for (const RhsState& s : h_state) {
      stats->iterations = std::max(stats->iterations, s.iters);
      stats->reliable_updates = std::max(stats->reliable_updates, s.ru);
      stats->converged += s.status == ST_DONE;
      const double res = s.bb > 0 ? std::sqrt(s.rr_true / s.bb) : 0.0;
      stats->true_residual = std::max(stats->true_residual, res);
    }
    stats->flops += hop_applications * (int64_t)1320 * ctx->g.n5h * nrhs;
  }

  int run(qdwf_solve_stats* stats) {
    int rc = begin();
    if (rc) return rc;
    for (;;) {
      bool fin = false;
      if ((rc = complete(&fin))) return rc;
      if (fin) break;
      if ((rc = launch())) return rc;
    }
    fill_stats(stats);
    return status;
  }
};

}  // namespace

namespace {

__global__ void __launch_bounds__(RT) k_axpby(double* __restrict__ out, const double* a, double ca,
                                              const double* b, double cb, long n, long rs_o,
                                              long rs_a, long rs_b) {
  const int q = blockIdx.y, NB = gridDim.x;
  for (long i = (long)blockIdx.x * RT + threadIdx.x; i < n; i += (long)NB * RT)
    out[(long)q * rs_o + i] = ca * a[(long)q * rs_a + i] + cb * b[(long)q * rs_b + i];
}

}  // namespace

int axpby64(double* out, const double* a, double ca, const double* b, double cb, long n,
            long rs_o, long rs_a, long rs_b, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(reduce_blocks(n), nrhs), dim3(RT), 0, st, out, a, ca, b, cb, n,
                     rs_o, rs_a, rs_b);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

size_t solve_ws_bytes(const qdwf_ctx* ctx, int inner, int nrhs, int system) {
  const long n = ctx->g.n5h * 24;
  size_t b = solver_layout(n, nrhs, inner, true).total;
  (void)system;
  return b;
}

// Normal-equation solve on odd half fields with stride n: M_pc^dag M_pc x = b.
static int solve_normal(qdwf_ctx* ctx, double* x, const double* b, int nrhs,
                        const qdwf_solve_params& prm, qdwf_solve_stats* stats, void* ws,
                        hipStream_t st, double tol) {
  const long n = ctx->g.n5h * 24;
  auto go = [&](auto stag, auto rtag) -> int {
    typedef decltype(stag) S;
    typedef decltype(rtag) R;
    Cg<S, R> cg;
    cg.ctx = ctx;
    cg.st = st;
    cg.layout = prm.layout;
    cg.inner = prm.inner_prec;
    cg.nrhs = nrhs;
    cg.n = n;
    cg.NB = reduce_blocks(n);
    cg.ws = reinterpret_cast<char*>(ws);
    cg.L = solver_layout(n, nrhs, prm.inner_prec, true);
    cg.xh = x;
    cg.rs_x = n;
    cg.b = b;
    cg.rs_b = n;
    const double delta = prm.delta > 0 ? prm.delta : 0.1;
    cg.delta2 = prm.inner_prec == QDWF_F64 ? 0.0 : delta * delta;
    cg.tol2 = tol * tol;
    cg.prm = prm;
    return cg.run(stats);
  };
  switch (prm.inner_prec) {
    case QDWF_F64: return go(double(), double());
    case QDWF_F32: return go(float(), float());
    case QDWF_F16: return go(_Float16(), float());
    case QDWF_BF16: return go(bf16(), float());
  }
  return fail(QDWF_EINVAL, "unknown inner precision %d", prm.inner_prec);
}

// Full system D x = b through the Schur complement on odd sites:
//   b'_o = b_o - M_oe M_ee^-1 b_e ; M_pc^dag M_pc x_o = M_pc^dag b'_o ;
//   x_e = M_ee^-1 (b_e - M_eo x_o).
// If |D x - b| / |b| is still above tol after the normal equations reach tol,
// they are solved again from the current x_o with a tenfold tighter target.
static int solve_full(qdwf_ctx* ctx, double* x, const double* b, int nrhs,
                      const qdwf_solve_params& prm, qdwf_solve_stats* stats, void* ws,
                      hipStream_t st) {
  const long n = ctx->g.n5h * 24;
  const Layout L = solver_layout(n, nrhs, prm.inner_prec, true);
  char* w = reinterpret_cast<char*>(ws);
  // FP64 scratch borrowed from the solver layout before the solve starts and
  // after it ends: rh, ax, vh, t1h, t2h, plus the two staging vectors.
  double* s_rhs = reinterpret_cast<double*>(w + L.off_stage);
  double* s_xo = s_rhs + n * nrhs;
  double* t1 = reinterpret_cast<double*>(w + L.off_t1h);
  double* t2 = reinterpret_cast<double*>(w + L.off_t2h);
  double* t3 = reinterpret_cast<double*>(w + L.off_vh);
  const long rs = 2 * n;                // full-field stride
  const double* be = b;                 // even half of each rhs
  const double* bo = b + n;
  double* xe = x;
  double* xo = x + n;
  int rc;
  auto hop = [&](int dag, int out_par, void* out, const void* in, long rs_io) {
    HopArgs a = {};
    a.in[out_par] = in;
    a.out[out_par] = out;
    a.rs_in = a.rs_out = a.rs_z = rs_io;
    a.par0 = out_par;
    a.npar = 1;
    a.nrhs = nrhs;
    a.hop_scale = -0.5;
    return launch_hop(ctx, QDWF_F64, prm.layout, dag, a, st);
  };
  // all FP64 half-field temporaries below have stride n; b and x halves stride 2n
  // t1 = b_e (copy, stride n), t2 = M_ee^-1 t1, t3 = M_oe t2, s_xo = b'_o = b_o - t3
  if ((rc = axpby64(t1, be, 1.0, be, 0.0, n, n, rs, rs, nrhs, st))) return rc;
  if ((rc = launch_local(ctx, QDWF_F64, prm.layout, MAT_MEEINV, t2, t1, 1, 0, n, nrhs, st))) return rc;
  if ((rc = hop(0, QDWF_ODD, t3, t2, n))) return rc;
  if ((rc = axpby64(s_xo, bo, 1.0, t3, -1.0, n, n, rs, n, nrhs, st))) return rc;
  // s_rhs = M_pc^dag b'_o
  if ((rc = apply_mpc(ctx, QDWF_F64, prm.layout, 1, s_rhs, s_xo, t1, t2, nrhs, n, st))) return rc;
  // initial guess: odd half of x (or zero)
  if (prm.x0_is_guess) {
    if ((rc = axpby64(s_xo, xo, 1.0, xo, 0.0, n, n, rs, rs, nrhs, st))) return rc;
  }
  qdwf_solve_params p2 = prm;
  double tol = prm.tol;
  int status = QDWF_OK;
  for (int round = 0; round < 4; ++round) {
    qdwf_solve_stats s1 = {};
    status = solve_normal(ctx, s_xo, s_rhs, nrhs, p2, &s1, ws, st, tol);
    if (stats) {
      stats->iterations += s1.iterations;
      stats->reliable_updates += s1.reliable_updates;
      stats->converged = s1.converged;
      stats->true_residual = s1.true_residual;
      stats->flops += s1.flops;
    }
    if (status != QDWF_OK) break;
    // x_o back into x; x_e = M_ee^-1 (b_e - M_eo x_o)
    if ((rc = axpby64(xo, s_xo, 1.0, s_xo, 0.0, n, rs, n, n, nrhs, st))) return rc;
    if ((rc = hop(0, QDWF_EVEN, t3, s_xo, n))) return rc;
    if ((rc = axpby64(t1, be, 1.0, t3, -1.0, n, n, rs, n, nrhs, st))) return rc;
    if ((rc = launch_local(ctx, QDWF_F64, prm.layout, MAT_MEEINV, t2, t1, 1, 0, n, nrhs, st))) return rc;
    if ((rc = axpby64(xe, t2, 1.0, t2, 0.0, n, rs, n, n, nrhs, st))) return rc;
    // full residual |D x - b| / |b| per rhs (D applied with the full-field hop)
    double* dx = reinterpret_cast<double*>(w + L.off_rh);   // 2n per rhs fits rh + ax
    HopArgs a = {};
    a.in[0] = x + n; a.in[1] = x;
    a.out[0] = dx; a.out[1] = dx + n;
    a.z[0] = x; a.z[1] = x + n;
    a.rs_in = rs; a.rs_out = rs; a.rs_z = rs;
    a.par0 = 0; a.npar = 2; a.nrhs = nrhs; a.epi = 1; a.hop_scale = -0.5;
    a.alpha = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
    a.beta = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
    if ((rc = launch_hop(ctx, QDWF_F64, prm.layout, 0, a, st))) return rc;
    // dx <- dx - b ; norms
    if ((rc = axpby64(dx, dx, 1.0, b, -1.0, 2 * n, rs, rs, rs, nrhs, st))) return rc;
    std::vector<double> rr(2 * nrhs), bb(2 * nrhs);
    void* dws = reinterpret_cast<void*>(w + L.off_part);
    // the partial buffer is large enough for one reduction over 2n reals per rhs
    if ((rc = dot_re_im(ctx, rr.data(), dx, dx, 2 * n, QDWF_F64, QDWF_RIRI, nrhs, dws, st))) return rc;
    if ((rc = dot_re_im(ctx, bb.data(), b, b, 2 * n, QDWF_F64, QDWF_RIRI, nrhs, dws, st))) return rc;
    double worst = 0;
    for (int q = 0; q < nrhs; ++q)
      worst = std::max(worst, bb[2 * q] > 0 ? std::sqrt(rr[2 * q] / bb[2 * q]) : 0.0);
    if (stats) stats->full_residual = worst;
    if (worst <= prm.tol) break;
    tol *= 0.1;
    p2.x0_is_guess = 1;
  }
  return status;
}

int solve(qdwf_ctx* ctx, double* x, const double* b, int nrhs, const qdwf_solve_params& prm,
          qdwf_solve_stats* stats, void* ws, hipStream_t st) {
  if (prm.system == QDWF_SYS_FULL) return solve_full(ctx, x, b, nrhs, prm, stats, ws, st);
  return solve_normal(ctx, x, b, nrhs, prm, stats, ws, st, prm.tol);
}

}  // namespace qdwf
