// Layout conversion between the canonical caller-facing arrays and the
// internal even-odd fields, and packing of the gauge links.
//
// Internal spinor half field (one parity): 5D site (i, s) where i is the
// site's index in the library's traversal order of that parity; the 24 reals
// of a site are interleaved complex, blocked over the Ls slices of a 4D site
// in chunks of 4 reals (RIRI), or split into 24 planes of length (V/2)*Ls
// ordered [re/im][spin][colour] (RRII); the offsets are in siteio.h.
// Links: [parity][mu][cb][18]
// (3x3 complex row-major, interleaved), with the boundary factor bc[mu]
// multiplied into U_mu(x) on the last slice x_mu = L_mu - 1, which is the one
// link used by both hops that cross that boundary.
#include "common.h"
#include "siteio.h"

namespace qdwf {

namespace {

// One thread per (rhs, half, 5D site of that half).
template <class R, class S, int LAYOUT, bool UNPACK>
__global__ void pack_kernel(const void* __restrict__ src_v, void* __restrict__ dst_v, int nhalf,
                            int par0, long n5h, int Ls, int V, const int* __restrict__ site_lex,
                            int Vh, int nrhs) {
  const long total = (long)nrhs * nhalf * n5h;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long j = idx % n5h;
    const long rh = idx / n5h;
    const int h = (int)(rh % nhalf);
    const int r = (int)(rh / nhalf);
    const int p = par0 + h;
    const int cb = (int)(j / Ls), s = (int)(j % Ls);
    const int lex = site_lex[(long)p * Vh + cb];
    const long cidx = (((long)r * Ls + s) * V + lex) * 24;   // canonical reals
    const long ibase = ((long)r * nhalf + h) * n5h * 24;     // internal half field
    if (!UNPACK) {
      const R* src = reinterpret_cast<const R*>(src_v) + cidx;
      S* dst = reinterpret_cast<S*>(dst_v) + ibase;
#pragma unroll
      for (int c = 0; c < 24; ++c) {
        const S v = Store<S>::from64((double)src[c]);
        if (LAYOUT == QDWF_RIRI) dst[riri_offset(cb, s, c, Ls)] = v;
        else dst[rrii_offset(cb, s, c, Ls, n5h)] = v;
      }
    } else {
      const S* src = reinterpret_cast<const S*>(src_v) + ibase;
      R* dst = reinterpret_cast<R*>(dst_v) + cidx;
#pragma unroll
      for (int c = 0; c < 24; ++c) {
        const S v = (LAYOUT == QDWF_RIRI) ? src[riri_offset(cb, s, c, Ls)]
                                          : src[rrii_offset(cb, s, c, Ls, n5h)];
        dst[c] = (R)Store<S>::to(v);
      }
    }
  }
}

template <class R, class S>
__global__ void link_kernel(const void* __restrict__ U_v, S* __restrict__ out, int Vh, int V,
                            const int* __restrict__ site_lex, int Lx, int Ly, int Lz, int Lt,
                            int bx, int by, int bz, int bt) {
  const long total = 2L * 4 * Vh;
  const R* U = reinterpret_cast<const R*>(U_v);
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int cb = (int)(idx % Vh);
    const int mu = (int)((idx / Vh) % 4);
    const int p = (int)(idx / (4L * Vh));
    const int lex = site_lex[(long)p * Vh + cb];
    int c[4];
    int rest = lex;
    c[0] = rest % Lx; rest /= Lx;
    c[1] = rest % Ly; rest /= Ly;
    c[2] = rest % Lz;
    c[3] = rest / Lz;
    const int Lm[4] = {Lx, Ly, Lz, Lt};
    const int bm[4] = {bx, by, bz, bt};
    const double f = (c[mu] == Lm[mu] - 1) ? (double)bm[mu] : 1.0;
    const R* src = U + ((long)mu * V + lex) * 18;
    S* dst = out + idx * 18;
#pragma unroll
    for (int k = 0; k < 18; ++k) dst[k] = Store<S>::from64((double)f * (double)src[k]);
  }
}

inline int grid_for(long n) {
  long b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int launch_pack(qdwf_ctx* ctx, void* dst, int prec, int layout, const void* src, int src_prec,
                int subset, int nrhs, hipStream_t st, bool unpack) {
  const Geom& g = ctx->g;
  const int nhalf = (subset == QDWF_FULL) ? 2 : 1;
  const int par0 = (subset == QDWF_ODD) ? 1 : 0;
  const long total = (long)nrhs * nhalf * g.n5h;
  auto go = [&](auto rtag, auto stag) -> int {
    typedef decltype(rtag) R;
    typedef decltype(stag) S;
    auto launch = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(grid_for(total)), dim3(256), 0, st, src, dst, nhalf, par0,
                         g.n5h, g.Ls, g.V, ctx->d_site_lex, g.Vh, nrhs);
    };
    // pack reads canonical (src) and writes internal (dst); unpack the reverse
    if (!unpack) {
      if (layout == QDWF_RIRI) launch(pack_kernel<R, S, QDWF_RIRI, false>);
      else launch(pack_kernel<R, S, QDWF_RRII, false>);
    } else {
      if (layout == QDWF_RIRI) launch(pack_kernel<R, S, QDWF_RIRI, true>);
      else launch(pack_kernel<R, S, QDWF_RRII, true>);
    }
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
  };
  auto by_s = [&](auto rtag) -> int {
    switch (prec) {
      case QDWF_F64: return go(rtag, double());
      case QDWF_F32: return go(rtag, float());
      case QDWF_F16: return go(rtag, _Float16());
      case QDWF_BF16: return go(rtag, bf16());
    }
    return fail(QDWF_EINVAL, "unknown precision %d", prec);
  };
  if (src_prec == QDWF_F64) return by_s(double());
  if (src_prec == QDWF_F32) return by_s(float());
  return fail(QDWF_EINVAL, "canonical spinors are complex128 (QDWF_F64) or complex64 (QDWF_F32)");
}

int launch_pack_links(qdwf_ctx* ctx, const void* U, int canon_prec, hipStream_t st) {
  const Geom& g = ctx->g;
  const int* bc = ctx->act.bc;
  const long total = 2L * 4 * g.Vh;
  auto go = [&](auto rtag, auto stag, void* out) -> int {
    typedef decltype(rtag) R;
    typedef decltype(stag) S;
    if (!out) return QDWF_OK;   // a precision this context does not keep
    hipLaunchKernelGGL((link_kernel<R, S>), dim3(grid_for(total)), dim3(256), 0, st, U,
                       reinterpret_cast<S*>(out), g.Vh, g.V, ctx->d_site_lex, g.L[0], g.L[1],
                       g.L[2], g.L[3],
                       bc[0], bc[1], bc[2], bc[3]);
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
  };
  auto all = [&](auto rtag) -> int {
    int rc;
    if ((rc = go(rtag, double(), ctx->d_links[QDWF_F64]))) return rc;
    if ((rc = go(rtag, float(), ctx->d_links[QDWF_F32]))) return rc;
    if ((rc = go(rtag, _Float16(), ctx->d_links[QDWF_F16]))) return rc;
    return go(rtag, bf16(), ctx->d_links[QDWF_BF16]);
  };
  if (canon_prec == QDWF_F64) return all(double());
  if (canon_prec == QDWF_F32) return all(float());
  return fail(QDWF_EINVAL, "canonical gauge field is complex128 (QDWF_F64) or complex64 (QDWF_F32)");
}

}  // namespace qdwf
