// The Wilson Dslash kernel (Section 4.1 names it beside the Domain Wall
// kernel; Table 1 measures it): the 4D hop D_h, optionally with the Wilson
// mass term, D_W = (4 + m) - D_h / 2.
//
// One lane per (5D site, rhs): for Ls = 1 a lane is one 4D site, for Ls > 1 the
// operator acts on every slice. Unlike the domain-wall kernel there is no
// reuse of links across the fifth dimension to exploit at Ls = 1, so each lane
// reads its 8 links straight from global memory and there is no LDS stage and
// no barrier. With Ls = 1 the links come from a lane-major copy built by
// qdwf_set_gauge: the 4 forward links of every site cut into chunks stored
// chunk-major over the sites, so that one load instruction of a wavefront
// reads consecutive words (5 loads per link instead of 9 narrow, strided
// ones); a backward link is read as its neighbour's forward link. With Ls > 1 the slices of a site
// share its links and the packed [parity][mu][site] links are read.
#include "common.h"
#include "siteio.h"
#include "spin.h"

namespace qdwf {

namespace {

// Lane-major links of Ls = 1 contexts: for each parity and direction mu,
// four chunks of 4 reals, each chunk-major over the sites ([c][site][4]),
// then the last 2 reals of every link ([site][2]): 18 reals per link, no
// padding, and consecutive lanes read consecutive words. Forward links only:
// the backward link U_mu(x - mu) is the forward link of the neighbour.
template <class S> struct WLinkIO {
  typedef typename Store<S>::compute T;
  __device__ static inline void load(const S* __restrict__ w, int p, int mu, int i, int Vh, T* U) {
    const S* base = w + ((long)p * 4 + mu) * Vh * 18;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const S* q = base + ((long)c * Vh + i) * 4;
      if constexpr (sizeof(S) == 8) {
        const double2 a = reinterpret_cast<const double2*>(q)[0];
        const double2 b = reinterpret_cast<const double2*>(q)[1];
        U[4 * c] = (T)a.x; U[4 * c + 1] = (T)a.y; U[4 * c + 2] = (T)b.x; U[4 * c + 3] = (T)b.y;
      } else if constexpr (sizeof(S) == 4) {
        const float4 a = *reinterpret_cast<const float4*>(q);
        U[4 * c] = (T)a.x; U[4 * c + 1] = (T)a.y; U[4 * c + 2] = (T)a.z; U[4 * c + 3] = (T)a.w;
      } else {
        const uint2 a = *reinterpret_cast<const uint2*>(q);
        S h[4];
        __builtin_memcpy(h, &a, 8);
#pragma unroll
        for (int e = 0; e < 4; ++e) U[4 * c + e] = Store<S>::to(h[e]);
      }
    }
    const S* q = base + (long)Vh * 16 + (long)i * 2;
    if constexpr (sizeof(S) == 8) {
      const double2 a = *reinterpret_cast<const double2*>(q);
      U[16] = (T)a.x; U[17] = (T)a.y;
    } else if constexpr (sizeof(S) == 4) {
      const float2 a = *reinterpret_cast<const float2*>(q);
      U[16] = (T)a.x; U[17] = (T)a.y;
    } else {
      const uint32_t a = *reinterpret_cast<const uint32_t*>(q);
      S h[2];
      __builtin_memcpy(h, &a, 4);
      U[16] = Store<S>::to(h[0]); U[17] = Store<S>::to(h[1]);
    }
  }
};

struct WilK {
  const void* in[2];
  void* out[2];
  const void* z[2];
  const void* links;   // [2][4][Vh][18] in the storage type, boundary factors folded in
  const void* wl;      // Ls = 1: lane-major links (see WLinkIO), else null
  const int* nbr;      // [2][8][Vh]
  long rs_in, rs_out, rs_z, plane;
  int Vh, Ls, nrhs, par0, npar, epi;
  double hop_scale, alpha;
};

template <class S, int LAYOUT, bool DAG, bool WL>
__global__ void __launch_bounds__(256) wilson_kernel(WilK k) {
  typedef typename Store<S>::compute T;
  const long n5 = (long)k.Vh * k.Ls;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= n5 * k.npar * k.nrhs) return;   // no barrier below
  const long j = tid % n5;
  const long rp = tid / n5;
  const int p = k.par0 + (int)(rp % k.npar);
  const int r = (int)(rp / k.npar);
  const int q = 1 - p;
  const int i = (int)(j / k.Ls), s = (int)(j - (long)i * k.Ls);
  const int Vh = k.Vh;
  const S* in = reinterpret_cast<const S*>(k.in[p]) + (long)r * k.rs_in;
  const S* lk = reinterpret_cast<const S*>(k.links);
  const int* nb = k.nbr + (long)p * 8 * Vh;

  T acc[24];
  auto step = [&](auto Dc) {
    constexpr int D = decltype(Dc)::value;
    constexpr int MU = D & 3;
    constexpr bool FWD = D < 4;
    // (1 - g) on forward hops and (1 + g) on backward ones; swapped for D_h^dag
    constexpr int SG = (FWD != DAG) ? -1 : +1;
    const int n = nb[(long)D * Vh + i];
    T v[24], U[18], h[12], uh[12];
    SiteIO<S, LAYOUT>::load(in, n, s, k.Ls, k.plane, v);
    if constexpr (WL) {
      // forward: U_mu(x) of this site; backward: U_mu(x - mu) of the neighbour
      WLinkIO<S>::load(reinterpret_cast<const S*>(k.wl), FWD ? p : q, MU, FWD ? i : n, Vh, U);
    } else {
      // forward: U_mu(x) of this site; backward: U_mu(x - mu) of the neighbour
      const long li = FWD ? (((long)p * 4 + MU) * Vh + i) : (((long)q * 4 + MU) * Vh + n);
      LinkIO<S>::load(lk + li * 18, U);
    }
    project<MU, SG>(v, h);
    su3_mul<!FWD>(U, h, uh);
    recon_acc<MU, SG, D == 0>(uh, acc);
  };
  step(IC<0>()); step(IC<1>()); step(IC<2>()); step(IC<3>());
  step(IC<4>()); step(IC<5>()); step(IC<6>()); step(IC<7>());

  const T hs = (T)k.hop_scale;
  if (k.epi) {
    const S* zf = reinterpret_cast<const S*>(k.z[p]) + (long)r * k.rs_z;
    T z[24];
    SiteIO<S, LAYOUT>::load(zf, i, s, k.Ls, k.plane, z);
    const T al = (T)k.alpha;
#pragma unroll
    for (int c = 0; c < 24; ++c) acc[c] = fmac(al, z[c], hs * acc[c]);
  } else {
#pragma unroll
    for (int c = 0; c < 24; ++c) acc[c] *= hs;
  }
  S* out = reinterpret_cast<S*>(k.out[p]) + (long)r * k.rs_out;
  SiteIO<S, LAYOUT>::store(out, i, s, k.Ls, k.plane, acc);
}

template <class S, int LAYOUT, bool DAG>
int run_wilson(qdwf_ctx* ctx, int prec, const HopArgs& a, hipStream_t st) {
  const Geom& g = ctx->g;
  WilK k;
  for (int h = 0; h < 2; ++h) { k.in[h] = a.in[h]; k.out[h] = a.out[h]; k.z[h] = a.z[h]; }
  k.links = ctx->d_links[prec];
  k.wl = (g.Ls == 1) ? ctx->d_wlinks[prec] : nullptr;
  k.nbr = ctx->d_nbr;
  k.rs_in = a.rs_in; k.rs_out = a.rs_out; k.rs_z = a.rs_z;
  k.plane = g.n5h;
  k.Vh = g.Vh; k.Ls = g.Ls; k.nrhs = a.nrhs; k.par0 = a.par0; k.npar = a.npar;
  k.epi = a.epi;
  k.hop_scale = a.hop_scale;
  k.alpha = a.alpha;
  const long total = g.n5h * a.npar * a.nrhs;
  const long blocks = (total + 255) / 256;
  if (blocks > 0x7fffffffL) return fail(QDWF_EINVAL, "problem too large for one launch");
  if (k.wl)
    hipLaunchKernelGGL((wilson_kernel<S, LAYOUT, DAG, true>), dim3((unsigned)blocks), dim3(256), 0, st, k);
  else
    hipLaunchKernelGGL((wilson_kernel<S, LAYOUT, DAG, false>), dim3((unsigned)blocks), dim3(256), 0, st, k);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

template <class S>
__global__ void wlink_kernel(const S* __restrict__ links, S* __restrict__ wl, int Vh) {
  const long total = 2L * 4 * Vh;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % Vh);
    const long pm = t / Vh;   // parity * 4 + mu, as in the packed links
    const S* src = links + t * 18;
    S* base = wl + pm * Vh * 18;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) base[((long)c * Vh + i) * 4 + e] = src[4 * c + e];
    base[(long)Vh * 16 + (long)i * 2] = src[16];
    base[(long)Vh * 16 + (long)i * 2 + 1] = src[17];
  }
}

}  // namespace

int launch_wilson_links(qdwf_ctx* ctx, hipStream_t st) {
  const Geom& g = ctx->g;
  const long total = 2L * 4 * g.Vh;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  auto go = [&](auto tag, int p) {
    typedef decltype(tag) S;
    hipLaunchKernelGGL(wlink_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const S*>(ctx->d_links[p]),
                       reinterpret_cast<S*>(ctx->d_wlinks[p]), g.Vh);
  };
  for (int p = QDWF_F64; p <= QDWF_BF16; ++p) {
    if (!ctx->d_wlinks[p]) continue;
    if (p == QDWF_F64) go(double(), p);
    else if (p == QDWF_F32) go(float(), p);
    else if (p == QDWF_F16) go(_Float16(), p);
    else go(bf16(), p);
    QDWF_HIP(hipGetLastError());
  }
  return QDWF_OK;
}

int launch_wilson(qdwf_ctx* ctx, int prec, int layout, int dagger, const HopArgs& a,
                  hipStream_t st) {
  auto go = [&](auto tag_s) -> int {
    typedef decltype(tag_s) S;
    if (layout == QDWF_RIRI)
      return dagger ? run_wilson<S, QDWF_RIRI, true>(ctx, prec, a, st)
                    : run_wilson<S, QDWF_RIRI, false>(ctx, prec, a, st);
    return dagger ? run_wilson<S, QDWF_RRII, true>(ctx, prec, a, st)
                  : run_wilson<S, QDWF_RRII, false>(ctx, prec, a, st);
  };
  switch (prec) {
    case QDWF_F64: return go(double());
    case QDWF_F32: return go(float());
    case QDWF_F16: return go(_Float16());
    case QDWF_BF16: return go(bf16());
  }
  return fail(QDWF_EINVAL, "unknown precision %d", prec);
}

}  // namespace qdwf
