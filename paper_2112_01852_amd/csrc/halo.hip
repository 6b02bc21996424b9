// Domain-decomposed domain-wall operator on one GPU: the lattice is cut into
// R slabs along t, as the paper's 4-rank runs cut a node's lattice between
// MPI ranks (Section 4.2, Tables 1 and 2), and D is applied the way a
// distributed run would apply it:
//   1. pack: every slab projects its two t-faces to half spinors, 12 reals
//      per face site and slice: (1 - g_t) A psi for the slab below (which
//      multiplies by its own link U_t), U_t^dag (1 + g_t) A psi for the slab
//      above (the link belongs to the sender);
//   2. exchange: the half spinors move between slabs (a device copy here,
//      where a multi-GPU run would send them over xGMI);
//   3. interior: the full hop kernel on local data, with the links that cross
//      a slab boundary zeroed so that no cross-slab hop contributes (it still
//      reads the neighbour spinor across the cut, which a distributed run
//      would not hold);
//   4. boundary: the face sites add the received hops.
// The result equals D up to the order of summation on the face sites.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "siteio.h"
#include "spin.h"

namespace qdwf {

namespace {

// Links with U_t zeroed on the top slice of every slab (the one link both
// hops across a slab boundary use).
template <class S>
__global__ void split_links_kernel(const S* __restrict__ src, S* __restrict__ dst, int Vh,
                                   const int* __restrict__ site_lex, int V3, int tslab) {
  const long n = (long)2 * 4 * Vh;
  for (long l = (long)blockIdx.x * blockDim.x + threadIdx.x; l < n;
       l += (long)gridDim.x * blockDim.x) {
    const int i = (int)(l % Vh);
    const int mu = (int)((l / Vh) % 4);
    const int p = (int)(l / ((long)4 * Vh));
    const int t = site_lex[(long)p * Vh + i] / V3;
    const bool cut = mu == 3 && (t % tslab) == tslab - 1;
    for (int c = 0; c < 18; ++c)
      dst[l * 18 + c] = cut ? Store<S>::from((typename Store<S>::compute)0) : src[l * 18 + c];
  }
}

// A face work item: slab r, face hi (0: first slice, 1: last), face site
// fx = (z*Ly + y)*Lx + x, slice s. Returns the site's parity and internal index.
struct FaceSite {
  int r, hi, s, p, i;
  long fx;
};
__device__ inline FaceSite face_site(long w, int Ls, int V3, int Lx, int Ly, int tslab,
                                     const int* __restrict__ idx) {
  FaceSite f;
  f.s = (int)(w % Ls);
  f.fx = (w / Ls) % V3;
  f.hi = (int)((w / ((long)Ls * V3)) % 2);
  f.r = (int)(w / ((long)Ls * V3 * 2));
  const int t = f.r * tslab + (f.hi ? tslab - 1 : 0);
  const int x = (int)(f.fx % Lx), y = (int)((f.fx / Lx) % Ly), z = (int)(f.fx / ((long)Lx * Ly));
  f.p = (x + y + z + t) & 1;
  f.i = idx[(long)t * V3 + f.fx];
  return f;
}

template <class S, int LAYOUT>
__global__ void halo_pack_kernel(const S* __restrict__ in, S* __restrict__ send_lo,
                                 S* __restrict__ send_hi, const S* __restrict__ links,
                                 const int* __restrict__ idx, int Vh, int Ls, long plane,
                                 long half, int V3, int Lx, int Ly, int tslab, int ranks,
                                 double b, double c, double mf) {
  typedef typename Store<S>::compute T;
  const long n = (long)ranks * 2 * V3 * Ls;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < n;
       w += (long)gridDim.x * blockDim.x) {
    const FaceSite f = face_site(w, Ls, V3, Lx, Ly, tslab, idx);
    const S* src = in + f.p * half;
    // chi = A psi = b psi + c (P- psi_{s+1} + P+ psi_{s-1}), walls -mf
    T v[24], up[24], dn[24], chi[24];
    SiteIO<S, LAYOUT>::load(src, f.i, f.s, Ls, plane, v);
    SiteIO<S, LAYOUT>::load(src, f.i, f.s + 1 < Ls ? f.s + 1 : 0, Ls, plane, up);
    SiteIO<S, LAYOUT>::load(src, f.i, f.s > 0 ? f.s - 1 : Ls - 1, Ls, plane, dn);
    const T cu = (f.s + 1 < Ls) ? (T)c : (T)(-mf * c);
    const T cd = (f.s > 0) ? (T)c : (T)(-mf * c);
#pragma unroll
    for (int k = 0; k < 12; ++k) chi[k] = fmac((T)b, v[k], cd * dn[k]);     // spins 0, 1: S_d
#pragma unroll
    for (int k = 12; k < 24; ++k) chi[k] = fmac((T)b, v[k], cu * up[k]);    // spins 2, 3: S_u
    T h[12], uh[12];
    S* dst;
    if (f.hi) {
      // for the slab above: U_t(x)^dag (1 + g_t) chi, x on this slab's last slice
      project<3, +1>(chi, h);
      T U[18];
      LinkIO<S>::load(links + (((long)f.p * 4 + 3) * Vh + f.i) * 18, U);
      su3_mul<true>(U, h, uh);
      dst = send_hi;
    } else {
      // for the slab below: (1 - g_t) chi; the receiver applies its own U_t
      project<3, -1>(chi, uh);
      dst = send_lo;
    }
    S* o = dst + (((long)f.r * V3 + f.fx) * Ls + f.s) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) o[k] = Store<S>::from(uh[k]);
  }
}

template <class S, int LAYOUT>
__global__ void halo_boundary_kernel(S* __restrict__ out, const S* __restrict__ recv_lo,
                                     const S* __restrict__ recv_hi, const S* __restrict__ links,
                                     const int* __restrict__ idx, int Vh, int Ls, long plane,
                                     long half, int V3, int Lx, int Ly, int tslab, int ranks,
                                     double hop_scale) {
  typedef typename Store<S>::compute T;
  const long n = (long)ranks * 2 * V3 * Ls;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < n;
       w += (long)gridDim.x * blockDim.x) {
    const FaceSite f = face_site(w, Ls, V3, Lx, Ly, tslab, idx);
    const S* src = (f.hi ? recv_hi : recv_lo) + (((long)f.r * V3 + f.fx) * Ls + f.s) * 12;
    T h[12], acc[24];
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] = Store<S>::to(src[k]);
    if (f.hi) {
      // from the slab above: (1 - g_t) U_t(x) chi(x + t)
      T U[18], uh[12];
      LinkIO<S>::load(links + (((long)f.p * 4 + 3) * Vh + f.i) * 18, U);
      su3_mul<false>(U, h, uh);
      recon_acc<3, -1, true>(uh, acc);
    } else {
      // from the slab below: (1 + g_t) U_t(x - t)^dag chi(x - t), multiplied there
      recon_acc<3, +1, true>(h, acc);
    }
    S* o = out + f.p * half;
    T v[24];
    SiteIO<S, LAYOUT>::load(o, f.i, f.s, Ls, plane, v);
    const T hs = (T)hop_scale;
#pragma unroll
    for (int k = 0; k < 24; ++k) v[k] = fmac(hs, acc[k], v[k]);
    SiteIO<S, LAYOUT>::store(o, f.i, f.s, Ls, plane, v);
  }
}

struct SplitLayout {
  size_t links, idx, face, total;   // byte offsets / sizes inside the workspace
};

SplitLayout split_layout(const qdwf_ctx* c, int ranks, int prec) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t rb = prec_bytes(prec);
  SplitLayout L;
  L.links = 0;
  L.idx = al((size_t)2 * 4 * c->g.Vh * 18 * rb);
  const size_t V3 = (size_t)c->g.L[0] * c->g.L[1] * c->g.L[2];
  L.face = L.idx + al(sizeof(int32_t) * (size_t)c->g.V);
  L.total = L.face + 4 * al((size_t)ranks * V3 * c->g.Ls * 12 * rb);   // send / receive, lo / hi
  return L;
}

size_t face_bytes(const qdwf_ctx* c, int ranks, int prec) {
  const size_t V3 = (size_t)c->g.L[0] * c->g.L[1] * c->g.L[2];
  return (((size_t)ranks * V3 * c->g.Ls * 12 * prec_bytes(prec)) + 255) & ~(size_t)255;
}

int check_split(const qdwf_ctx* c, int ranks, int prec) {
  if (!c) return fail(QDWF_EINVAL, "null context");
  if (prec < QDWF_F64 || prec > QDWF_BF16) return fail(QDWF_EINVAL, "unknown precision %d", prec);
  if (ranks < 1 || c->g.L[3] % ranks != 0 || c->g.L[3] / ranks < 2)
    return fail(QDWF_EINVAL, "ranks = %d must divide Lt = %d into slabs of at least 2 slices",
                ranks, c->g.L[3]);
  return QDWF_OK;
}

int grid_for(long n) { return (int)std::min<long>((n + 255) / 256, 65536L); }

// f(S()) with S the storage type of `prec`
template <class F> int by_prec(int prec, F&& f) {
  switch (prec) {
    case QDWF_F64: return f(double());
    case QDWF_F32: return f(float());
    case QDWF_F16: return f(_Float16());
    case QDWF_BF16: return f(bf16());
  }
  return fail(QDWF_EINVAL, "unknown precision %d", prec);
}

}  // namespace

}  // namespace qdwf

using namespace qdwf;

extern "C" {

size_t qdwf_split_workspace_bytes(const qdwf_ctx* ctx, int ranks, int prec) {
  if (check_split(ctx, ranks, prec) != QDWF_OK) return 0;
  return split_layout(ctx, ranks, prec).total;
}

int qdwf_split_prepare(qdwf_ctx* ctx, int ranks, int prec, void* ws, void* stream) {
  if (int rc = check_split(ctx, ranks, prec)) return rc;
  if (!ws) return fail(QDWF_EINVAL, "ws is NULL");
  if (!ctx->gauge_set) return fail(QDWF_EINVAL, "gauge field not set (call qdwf_set_gauge first)");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const SplitLayout L = split_layout(ctx, ranks, prec);
  char* w = reinterpret_cast<char*>(ws);
  const int V3 = ctx->g.L[0] * ctx->g.L[1] * ctx->g.L[2];
  const int tslab = ctx->g.L[3] / ranks;
  int rc = by_prec(prec, [&](auto tag) -> int {
    typedef decltype(tag) S;
    hipLaunchKernelGGL(split_links_kernel<S>, dim3(grid_for((long)8 * ctx->g.Vh)), dim3(256), 0, st,
                       reinterpret_cast<const S*>(ctx->d_links[prec]),
                       reinterpret_cast<S*>(w + L.links), ctx->g.Vh, ctx->d_site_lex, V3, tslab);
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
  });
  if (rc == QDWF_OK) {
    const hipError_t e = hipMemcpyAsync(w + L.idx, ctx->geo->idx.data(), sizeof(int32_t) * ctx->g.V,
                                        hipMemcpyHostToDevice, st);
    if (e == hipSuccess) (void)hipStreamSynchronize(st);
    else rc = fail(QDWF_EDEVICE, "hipMemcpyAsync failed: %s", hipGetErrorString(e));
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc == QDWF_OK) set_error("");
  return rc;
}

int qdwf_apply_D_split(qdwf_ctx* ctx, void* out, const void* in, int ranks, int prec,
                       int layout, void* ws, void* stream) {
  if (int rc = check_split(ctx, ranks, prec)) return rc;
  if (!out || !in || !ws) return fail(QDWF_EINVAL, "null argument");
  if (out == in) return fail(QDWF_EINVAL, "out must not alias in");
  if (layout != QDWF_RIRI && layout != QDWF_RRII) return fail(QDWF_EINVAL, "unknown layout %d", layout);
  if (!ctx->gauge_set) return fail(QDWF_EINVAL, "gauge field not set (call qdwf_set_gauge first)");
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Geom& g = ctx->g;
  const SplitLayout L = split_layout(ctx, ranks, prec);
  const size_t fb = face_bytes(ctx, ranks, prec);
  char* w = reinterpret_cast<char*>(ws);
  char* send_lo = w + L.face;
  char* send_hi = send_lo + fb;
  char* recv_lo = send_hi + fb;
  char* recv_hi = recv_lo + fb;
  const int* idx = reinterpret_cast<const int*>(w + L.idx);
  const int V3 = g.L[0] * g.L[1] * g.L[2];
  const int tslab = g.L[3] / ranks;
  const long half = g.n5h * 24;
  const long nface = (long)ranks * 2 * V3 * g.Ls;
  const size_t slab_bytes = (size_t)V3 * g.Ls * 12 * prec_bytes(prec);
  const double al = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
  const double be = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
  int rc = by_prec(prec, [&](auto tag) -> int {
    typedef decltype(tag) S;
    const S* lk = reinterpret_cast<const S*>(ctx->d_links[prec]);
    // 1. pack both faces of every slab
    auto pack = [&](auto lay) {
      constexpr int LAY = decltype(lay)::value;
      hipLaunchKernelGGL((halo_pack_kernel<S, LAY>), dim3(grid_for(nface)), dim3(256), 0, st,
                         reinterpret_cast<const S*>(in), reinterpret_cast<S*>(send_lo),
                         reinterpret_cast<S*>(send_hi), lk, idx, g.Vh, g.Ls, g.n5h, half, V3,
                         g.L[0], g.L[1], tslab, ranks, ctx->act.b, ctx->act.c, ctx->act.mf);
    };
    if (layout == QDWF_RIRI) pack(IC<QDWF_RIRI>()); else pack(IC<QDWF_RRII>());
    QDWF_HIP(hipGetLastError());
    // 2. exchange: slab r receives slab r-1's top face and slab r+1's bottom face
    QDWF_HIP(hipMemcpyAsync(recv_lo + slab_bytes, send_hi, slab_bytes * (ranks - 1),
                            hipMemcpyDeviceToDevice, st));
    QDWF_HIP(hipMemcpyAsync(recv_lo, send_hi + slab_bytes * (ranks - 1), slab_bytes,
                            hipMemcpyDeviceToDevice, st));
    QDWF_HIP(hipMemcpyAsync(recv_hi, send_lo + slab_bytes, slab_bytes * (ranks - 1),
                            hipMemcpyDeviceToDevice, st));
    QDWF_HIP(hipMemcpyAsync(recv_hi + slab_bytes * (ranks - 1), send_lo, slab_bytes,
                            hipMemcpyDeviceToDevice, st));
    // 3. interior: D with the cross-slab links zeroed
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
    a.nrhs = 1;
    a.epi = 1;
    a.hop_scale = -0.5;
    a.alpha = al;
    a.beta = be;
    a.links = w + L.links;
    if (int r2 = launch_hop(ctx, prec, layout, 0, a, st)) return r2;
    // 4. boundary: add the received hops on the face sites
    auto bnd = [&](auto lay) {
      constexpr int LAY = decltype(lay)::value;
      hipLaunchKernelGGL((halo_boundary_kernel<S, LAY>), dim3(grid_for(nface)), dim3(256), 0, st,
                         reinterpret_cast<S*>(out), reinterpret_cast<const S*>(recv_lo),
                         reinterpret_cast<const S*>(recv_hi), lk, idx, g.Vh, g.Ls, g.n5h, half,
                         V3, g.L[0], g.L[1], tslab, ranks, -0.5);
    };
    if (layout == QDWF_RIRI) bnd(IC<QDWF_RIRI>()); else bnd(IC<QDWF_RRII>());
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
  });
  if (prev >= 0) (void)hipSetDevice(prev);
  if (rc == QDWF_OK) set_error("");
  return rc;
}

}  // extern "C"
