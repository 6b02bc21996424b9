// The Wilson Dslash kernel (Section 4.1 names it beside the Domain Wall
// kernel; Table 1 measures it): the 4D hop D_h, optionally with the Wilson
// mass term, D_W = (4 + m) - D_h / 2.
//
// One lane per (5D site, rhs): for Ls = 1 a lane is one 4D site, for Ls > 1 the
// operator acts on every slice. Unlike the domain-wall kernel there is no
// reuse of links across the fifth dimension to exploit at Ls = 1, so each lane
// reads its 8 links straight from global memory (4 forward links of its own
// site, which consecutive lanes read contiguously, and 4 backward links of its
// neighbours) and there is no LDS stage and no barrier.
#include "common.h"
#include "siteio.h"
#include "spin.h"

namespace qdwf {

namespace {

struct WilK {
  const void* in[2];
  void* out[2];
  const void* z[2];
  const void* links;   // [2][4][Vh][18] in the storage type, boundary factors folded in
  const int* nbr;      // [2][8][Vh]
  long rs_in, rs_out, rs_z, plane;
  int Vh, Ls, nrhs, par0, npar, epi;
  double hop_scale, alpha;
};

template <class S, int LAYOUT, bool DAG>
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
    // forward: U_mu(x) of this site; backward: U_mu(x - mu) of the neighbour
    const long li = FWD ? (((long)p * 4 + MU) * Vh + i) : (((long)q * 4 + MU) * Vh + n);
    LinkIO<S>::load(lk + li * 18, U);
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
  hipLaunchKernelGGL((wilson_kernel<S, LAYOUT, DAG>), dim3((unsigned)blocks), dim3(256), 0, st, k);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

}  // namespace

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
