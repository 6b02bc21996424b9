// The Domain Wall kernel's body, shared by the launch over one context
// (hop.hip) and the grouped launch over many contexts (group.hip): the 4D
// Wilson hop D_h applied on every slice of the fifth dimension (the kernel
// Section 4.1 measures; 1320 flops per 5D site in Table 3), fused with the
// Mobius 5D factors and the 4D-local epilogue so that one pass over memory
// gives D, D^dag, M_pq, (M_qp)^dag, or the last stage of M_pc / M_pc^dag.
//
// Work decomposition (one lane per 5D site and right-hand side):
//   * a wavefront holds floor(64/Ls) groups of Ls lanes; the lanes of a group
//     are the Ls slices of one (4D site, rhs) pair, so the s +- 1 neighbours
//     needed by the 5D operator C live in the same wavefront and are fetched
//     with cross-lane permutes instead of memory reloads;
//   * a block covers nsb consecutive checkerboard sites times nrb right-hand
//     sides; the 8 links of each of its 4D sites (4 forward U_mu(x), 4 backward
//     U_mu(x-mu)) are staged once in LDS and shared by all Ls*nrb lanes of the
//     site (Section 4.2 credits the Domain Wall kernel's advantage over Wilson
//     Dslash to exactly this reuse of links across the fifth dimension);
//   * the spin projection (1 -+ g_mu) reduces each neighbour spinor to a
//     half spinor before the SU(3) multiply, so only 2 colour vectors are
//     multiplied per direction (Table 3 counts this as 1320 flops per site).
#pragma once

#include <type_traits>

#include "cgtypes.h"
#include "common.h"
#include "hopcore.h"
#include "pk16.h"
#include "siteio.h"
#include "spin.h"

namespace qdwf {

struct HopK {
  const void* in[2];
  void* out[2];
  const void* z[2];
  const void* links;   // [2][4][Vh][18] in the storage type
  const int* nbr;      // [2][8][Vh]
  long rs_in, rs_out, rs_z, plane;
  int Vh, Ls, nrhs, par0, npar;
  int nsb, nrb, gpw, nrblk;
  int epi, xcd, minv;
  double c_over_b, mf, hop_scale_b, alpha, beta;
  double rpow[4];      // (-beta/alpha)^(2^j), j < 4: the M_ee^-1 scan
  const int* skip;     // per-rhs skip flags (HopArgs::skip), or nullptr
  int skip_stride;
  int cg;              // fused CG step (HopArgs::cg)
  void* cg_r;
  const double* cg_alpha;
  int cg_alpha_stride;
  double* cg_site;
  void* cg_x;          // cg = 3: inner solution, compute type
  const void* cg_p;    // cg = 3: search direction, storage type
};

// Target occupancy (waves per SIMD) the register allocator plans for: two for
// 32- and 64-bit storage, whose arithmetic needs the registers to keep two
// directions' neighbour loads in flight (the one-parity FP32 launches of
// hop.hip take three instead); four for the packed FP16 path
// (interleaved layout, Ls = 16: neighbour spinors stay packed, 105-114
// registers, no spills), three for other 16-bit storage (which spills at
// four).
template <class S, int LAYOUT = QDWF_RRII, bool DPP16 = false> struct WavesPerEU {
  static constexpr int v =
      sizeof(S) >= 4 ? 2 : (std::is_same<S, _Float16>::value && LAYOUT == QDWF_RIRI && DPP16) ? 4 : 3;
};

// The 18 words of a link staged in LDS in its two sign-adjusted forms
// (link_words), read as four 16-byte and one 8-byte LDS loads.
__device__ inline void load_link_words(const float* p, uint32_t* U) {
  const uint4* q4 = reinterpret_cast<const uint4*>(p);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint4 t4 = q4[j];
    U[4 * j] = t4.x; U[4 * j + 1] = t4.y; U[4 * j + 2] = t4.z; U[4 * j + 3] = t4.w;
  }
  const uint2 t2 = reinterpret_cast<const uint2*>(p)[8];
  U[16] = t2.x; U[17] = t2.y;
}

// One block's share of a hop launch: logical block L of the launch described
// by k (its sites, parity and right-hand sides), with smem the block's LDS
// (the LDS bytes make_hopk reports). Every 5D site's result depends only on
// k and the site, not on which block or launch computes it.
// CHI (D_h only, not the adjoint): without MINV the input already holds
// chi = (A/b) psi, so the hop takes it as it is; with MINV the result is
// multiplied by A/b after M_ee^-1 (the two commute: both are functions of
// C), so that the next hop of M_pc can take it as chi.
// FP16 storage in the interleaved layout takes the packed path (pk16.h):
// neighbour spinors stay packed, half spinors are projected in packed FP16
// and multiplied with v_dot2_f32_f16 into FP32. BF16 storage in that layout
// projects in FP32 and multiplies with v_dot2_f32_bf16 (no packed BF16 adds
// on this hardware).
template <class S, int LAYOUT, bool DAG, bool DPP16, bool MINV, bool CHI = false>
__device__ inline void hop_block(const HopK& k, int L, unsigned char* smem) {
  typedef typename Store<S>::compute T;
  static_assert(!(DAG && CHI), "the adjoint hop applies A^dag once per site");
  constexpr bool PK = std::is_same<S, _Float16>::value && LAYOUT == QDWF_RIRI;
  // BF16 storage, interleaved: FP32 spinor arithmetic, SU(3) products as
  // v_dot2_f32_bf16 on the half spinor rounded to BF16 and the packed links
  constexpr bool PKB = std::is_same<S, bf16>::value && LAYOUT == QDWF_RIRI;
  constexpr int LSTR = LinkStride<T>::v;
  T* su = reinterpret_cast<T*>(smem);                       // [nsb][8][LSTR]
  int* snb = reinterpret_cast<int*>(su + (size_t)8 * LSTR * k.nsb);   // [8][nsb]

  // logical block L: parity fastest, then sites, then right-hand-side
  // blocks, so the right-hand sides sweep the lattice one after another and
  // the working set the caches see is one field at a time
  const int nsblk = (k.Vh + k.nsb - 1) / k.nsb;
  const int p = k.par0 + L % k.npar;
  const int t1 = L / k.npar;
  const int sb = t1 % nsblk;
  const int rb = t1 / nsblk;
  const int q = 1 - p;
  const int cb0 = sb * k.nsb;
  const int Vh = k.Vh;
  if (k.skip) {
    // the whole block returns (before any barrier) when none of its
    // right-hand sides is running
    bool run = false;
    for (int j = 0; j < k.nrb; ++j) {
      const int r = rb * k.nrb + j;
      if (r < k.nrhs && k.skip[(long)r * k.skip_stride] == 0) run = true;
    }
    if (!run) return;
  }

  // Stage the neighbour indices of the block's sites (one load per thread),
  // then start this lane's first two neighbour-spinor loads, then stage the
  // links with every load of this thread in flight at once, so the block pays
  // about two memory latencies before its arithmetic starts.
  const int* nbp = k.nbr + (long)p * 8 * Vh;
  for (int i = threadIdx.x; i < 8 * k.nsb; i += blockDim.x) {
    const int d = i / k.nsb, sl = i - d * k.nsb;
    const int cb = min(cb0 + sl, Vh - 1);
    snb[i] = nbp[(long)d * Vh + cb];
  }
  __syncthreads();

  const int Ls = DPP16 ? 16 : k.Ls;   // a constant on the Ls = 16 path
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane / Ls, s = lane - gl * Ls;
  const bool lane_ok = gl < k.gpw;
  const int gid = wave * k.gpw + (lane_ok ? gl : 0);
  const int sl = gid / k.nrb, rl = gid - sl * k.nrb;
  const int cb = cb0 + sl, r = rb * k.nrb + rl;
  const bool active = lane_ok && cb < Vh && r < k.nrhs;
  const int rc = min(r, k.nrhs - 1);
  const int cbc = min(cb, Vh - 1);
  const S* in = reinterpret_cast<const S*>(k.in[p]) + (long)rc * k.rs_in;
  const int* nbs = snb + sl;

  // two neighbour spinors in flight (packed path: 12 words each)
  T va[24], vb[24];
  uint32_t wa[12], wb[12];
  // a site's 24 reals as 12 (re, im) FP16 words, in the order of SiteIO
  auto load_pk = [&](int site, uint32_t* w) {
    long i = site;
    int ss = s, lsb = Ls;
    riri_block(i, ss, lsb);
    const uint2* pp = reinterpret_cast<const uint2*>(in + i * lsb * 24 + (long)ss * 4);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const uint2 qq = pp[c * lsb];
      w[2 * c] = qq.x;
      w[2 * c + 1] = qq.y;
    }
  };
  if constexpr (PK) {
    load_pk(nbs[0], wa);
    load_pk(nbs[k.nsb], wb);
  } else {
    SiteIO<S, LAYOUT>::load(in, nbs[0], s, Ls, k.plane, va);
    SiteIO<S, LAYOUT>::load(in, nbs[k.nsb], s, Ls, k.plane, vb);
  }

  {
    // one thread per link: 18 contiguous reals, loaded with vector loads
    // (packed path: 9 (re, im) words, staged in the two sign-adjusted forms
    // of link_words)
    const S* lk = reinterpret_cast<const S*>(k.links);
    const int nlink = 8 * k.nsb;
    for (int i = threadIdx.x; i < nlink; i += blockDim.x) {
      const int d = i / k.nsb, sl2 = i - d * k.nsb;
      const int mu = d & 3;
      int par, site;
      if (d < 4) { par = p; site = min(cb0 + sl2, Vh - 1); }
      else       { par = q; site = snb[d * k.nsb + sl2]; }
      const S* src = lk + (((long)par * 4 + mu) * Vh + site) * 18;
      if constexpr (PK || PKB) {
        const uint32_t* qw = reinterpret_cast<const uint32_t*>(src);
        uint32_t* dstw = reinterpret_cast<uint32_t*>(su + (sl2 * 8 + d) * LSTR);
        uint32_t w[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) w[c] = qw[c];
#pragma unroll
        for (int c = 0; c < 9; ++c) link_words(w[c], d < 4, &dstw[c], &dstw[9 + c]);
      } else {
        T Ul[18];
        LinkIO<S>::load(src, Ul);
        T* dstp = su + (sl2 * 8 + d) * LSTR;
#pragma unroll
        for (int c = 0; c < 18; ++c) dstp[c] = Ul[c];
      }
    }
  }
  __syncthreads();

  const int base = gl * Ls;
  SShift<DPP16> sh;
  sh.src_m = lane_ok ? base + (s == 0 ? Ls - 1 : s - 1) : lane;   // holds slice s-1
  sh.src_p = lane_ok ? base + (s == Ls - 1 ? 0 : s + 1) : lane;   // holds slice s+1
  const T mf = (T)k.mf;
  const T wm = (s == 0) ? -mf : (T)1;        // wall factor of S_d at this slice
  const T wp = (s == Ls - 1) ? -mf : (T)1;   // wall factor of S_u at this slice
  // A = b (1 + (c/b) C); the factor b is applied once at the end
  const T cb_ = (T)k.c_over_b;
  const T cm = cb_ * wm, cp = cb_ * wp;
  const T* lks = su + sl * 8 * LSTR;
  // the same factors as FP16 pairs, for the packed path's A
  const uint32_t cmh = PK ? pk_f16((float)cm, (float)cm) : 0u;
  const uint32_t cph = PK ? pk_f16((float)cp, (float)cp) : 0u;

  T acc[24];
  // direction D uses the buffer loaded two steps earlier and refills it with
  // direction D + 2
  auto step = [&](auto Dc) {
    constexpr int D = decltype(Dc)::value;
    constexpr int MU = D & 3;
    constexpr bool FWD = D < 4;
    // (1 - g) on forward hops and (1 + g) on backward ones; swapped for D_h^dag
    constexpr int SG = (FWD != DAG) ? -1 : +1;
    // chi / b = psi + (c/b) (P+ psi_{s-1} + P- psi_{s+1}), walls included,
    // unless the input already holds it (CHI without MINV) or the hop is the
    // adjoint's
    constexpr bool APPLY_A = !DAG && !(CHI && !MINV);
    T uh[12];
    if constexpr (PK) {
      uint32_t* buf = (D & 1) ? wb : wa;
      uint32_t w[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) w[i] = buf[i];
      if constexpr (D < 6) load_pk(nbs[(D + 2) * k.nsb], buf);
      uint32_t h[6];
      if constexpr (APPLY_A) {
        // chi / b = psi + (c/b) (P+ psi_{s-1} + P- psi_{s+1}) in packed FP16:
        // upper spins (words 0-5) from slice s-1, lower (6-11) from s+1 (a
        // DPP row rotate at Ls = 16, a cross-lane permute otherwise)
        auto from_m = [&](uint32_t v) -> uint32_t {
          if constexpr (DPP16) return (uint32_t)dpp_ror<1>((int)v);
          else return (uint32_t)__shfl((int)v, sh.src_m, 64);
        };
        auto from_p = [&](uint32_t v) -> uint32_t {
          if constexpr (DPP16) return (uint32_t)dpp_ror<15>((int)v);
          else return (uint32_t)__shfl((int)v, sh.src_p, 64);
        };
        uint32_t x[12];
#pragma unroll
        for (int i = 0; i < 12; ++i)
          x[i] = i < 6 ? pk_fma(cmh, from_m(w[i]), w[i]) : pk_fma(cph, from_p(w[i]), w[i]);
        project_pk<MU, SG>(x, h);
      } else {
        project_pk<MU, SG>(w, h);
      }
      uint32_t U[18];
      load_link_words(lks + D * LSTR, U);
      su3_mul_pk<!FWD>(U, U + 9, h, uh);
    } else {
      T* buf = (D & 1) ? vb : va;
      T v[24];
#pragma unroll
      for (int i = 0; i < 24; ++i) v[i] = buf[i];
      if constexpr (D < 6)
        SiteIO<S, LAYOUT>::load(in, nbs[(D + 2) * k.nsb], s, Ls, k.plane, buf);
      if constexpr (APPLY_A) {
        T w[24];
#pragma unroll
        for (int i = 0; i < 24; ++i) w[i] = v[i];
        shift_s<1, 15>(sh, cm, cp, w, v);
      }
      T h[12];
      project<MU, SG>(v, h);
      if constexpr (PKB) {
        uint32_t hw[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) hw[i] = pk_bf16(h[2 * i], h[2 * i + 1]);
        uint32_t U[18];
        load_link_words(lks + D * LSTR, U);
        su3_mul_pk<!FWD, true>(U, U + 9, hw, uh);
      } else {
        T U[18];
        load_link(lks + D * LSTR, U);
        su3_mul<!FWD>(U, h, uh);
      }
    }
    recon_acc<MU, SG, D == 0>(uh, acc);
  };
  step(IC<0>()); step(IC<1>()); step(IC<2>()); step(IC<3>());
  step(IC<4>()); step(IC<5>()); step(IC<6>()); step(IC<7>());

  if constexpr (DAG) {
    // A^dag h / b = h + (c/b) C^dag h, C^dag = P- S_d + P+ S_u:
    // upper spins come from s+1, lower spins from s-1
    T tmp[24];
#pragma unroll
    for (int i = 0; i < 24; ++i) tmp[i] = acc[i];
    shift_s<15, 1>(sh, cp, cm, acc, tmp);
#pragma unroll
    for (int i = 0; i < 24; ++i) acc[i] = tmp[i];
  }
  if constexpr (MINV) {
    {
      // out = M_ee^-1 (or M_ee^-dag) applied to the hop result, across the 16
      // slices of the row: (alpha + beta S)^-1 on each chirality is a cyclic
      // geometric series in S, summed by doubling (steps 1, 2, 4, 8), with -mf
      // on the terms that wrap; its common factor is folded into the scale.
      // M_ee: upper spins see S_d (slice s - d), lower spins S_u (s + d);
      // the adjoint swaps them.
      auto scan = [&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        constexpr int Dd = 1 << J;
        const T rp = (T)k.rpow[J];
        const T cdn = (s - Dd < 0) ? rp * (-mf) : rp;    // source slice s - d
        const T cup = (s + Dd >= 16) ? rp * (-mf) : rp;  // source slice s + d
        T src[24];
#pragma unroll
        for (int i = 0; i < 24; ++i) src[i] = acc[i];
        if constexpr (DAG) shift_s<16 - Dd, Dd>(sh, cup, cdn, src, acc);
        else shift_s<Dd, 16 - Dd>(sh, cdn, cup, src, acc);
      };
      scan(IC<0>()); scan(IC<1>()); scan(IC<2>()); scan(IC<3>());
    }
    if constexpr (CHI) {
      // chi / b of the result for the next hop: (1 + (c/b) C) M_ee^-1 h
      T tmp[24];
#pragma unroll
      for (int i = 0; i < 24; ++i) tmp[i] = acc[i];
      shift_s<1, 15>(sh, cm, cp, tmp, acc);
    }
  }
  const T hs = (T)k.hop_scale_b;   // hop scale times b (and the M_ee^-1 factor)
  if (k.epi) {
    const S* zf = reinterpret_cast<const S*>(k.z[p]) + (long)rc * k.rs_z;
    T z[24];
    SiteIO<S, LAYOUT>::load(zf, cbc, s, Ls, k.plane, z);
    const T al = (T)k.alpha, be = (T)k.beta;
    const T bm = be * wm, bp = be * wp;
#pragma unroll
    for (int i = 0; i < 24; ++i) acc[i] = fmac(al, z[i], hs * acc[i]);
    if constexpr (!DAG) shift_s<1, 15>(sh, bm, bp, z, acc);   // + beta C z
    else shift_s<15, 1>(sh, bp, bm, z, acc);                  // + beta C^dag z
  } else {
#pragma unroll
    for (int i = 0; i < 24; ++i) acc[i] *= hs;
  }
  if (active && k.cg < 2) {
    S* out = reinterpret_cast<S*>(k.out[p]) + (long)rc * k.rs_out;
    if constexpr (PK) {
      long i = cbc;
      int ss = s, lsb = Ls;
      riri_block(i, ss, lsb);
      uint2* pp = reinterpret_cast<uint2*>(out + i * lsb * 24 + (long)ss * 4);
#pragma unroll
      for (int c = 0; c < 6; ++c)
        pp[c * lsb] = make_uint2(pk_f16(acc[4 * c], acc[4 * c + 1]), pk_f16(acc[4 * c + 2], acc[4 * c + 3]));
    } else {
      SiteIO<S, LAYOUT>::store(out, cbc, s, Ls, k.plane, acc);
    }
  }
  if (!MINV && k.cg) {
    // the CG step: this 5D site's sum of squares (components in order), then
    // each checkerboard site's sum over its slices in slice order (FP64), so
    // the per-site values do not depend on the launch shape. The site's sum
    // is taken in FP32 where the values are 16-bit numbers as stored (their
    // squares are exact in FP32, and 24 of them add with a relative error
    // below 2^-19), in FP64 otherwise.
    const bool live = active && (!k.skip || k.skip[(long)rc * k.skip_stride] == 0);
    double ss = 0.0;
    if (k.cg == 1) {
      if constexpr (sizeof(S) == 2) {
        float s32 = 0.0f;
#pragma unroll
        for (int i = 0; i < 24; ++i) {
          const float v = (float)Store<S>::to(Store<S>::from(acc[i]));   // as stored
          s32 = __builtin_fmaf(v, v, s32);
        }
        ss = (double)s32;
      } else {
#pragma unroll
        for (int i = 0; i < 24; ++i) {
          const double v = (double)Store<S>::to(Store<S>::from(acc[i]));   // as stored
          ss += v * v;
        }
      }
    } else if (live) {
      typedef typename ResidStore<S>::t RS;
      RS* rr = reinterpret_cast<RS*>(k.cg_r) + (long)rc * k.rs_out;
      T rv[24];
      SiteIO<RS, LAYOUT>::load(rr, cbc, s, Ls, k.plane, rv);
      const T al = (T)k.cg_alpha[(long)rc * k.cg_alpha_stride];
      if constexpr (sizeof(RS) == 2) {
        float s32 = 0.0f;
#pragma unroll
        for (int i = 0; i < 24; ++i) {
          rv[i] = rv[i] - al * acc[i];
          const float v = (float)Store<RS>::to(Store<RS>::from(rv[i]));   // as stored
          s32 = __builtin_fmaf(v, v, s32);
        }
        ss = (double)s32;
      } else {
#pragma unroll
        for (int i = 0; i < 24; ++i) {
          rv[i] = rv[i] - al * acc[i];
          const double v = (double)Store<RS>::to(Store<RS>::from(rv[i]));   // as stored
          ss += v * v;
        }
      }
      SiteIO<RS, LAYOUT>::store(rr, cbc, s, Ls, k.plane, rv);
      if (k.cg == 3) {
        // the iteration's step at the same sites: x += alpha p
        T pv[24], xv[24];
        SiteIO<S, LAYOUT>::load(reinterpret_cast<const S*>(k.cg_p) + (long)rc * k.rs_out, cbc, s,
                                Ls, k.plane, pv);
        T* xr = reinterpret_cast<T*>(k.cg_x) + (long)rc * k.rs_out;
        SiteIO<T, LAYOUT>::load(xr, cbc, s, Ls, k.plane, xv);
#pragma unroll
        for (int i = 0; i < 24; ++i) xv[i] = xv[i] + al * pv[i];
        SiteIO<T, LAYOUT>::store(xr, cbc, s, Ls, k.plane, xv);
      }
    }
    double* red = reinterpret_cast<double*>(snb + 8 * k.nsb);   // blockDim.x doubles
    red[threadIdx.x] = live ? ss : 0.0;
    __syncthreads();
    if (live && s == 0) {
      double t = 0.0;
      for (int j = 0; j < Ls; ++j) t += red[threadIdx.x + j];
      k.cg_site[(long)rc * Vh + cb] = t;
    }
  }
}


// Kernel arguments of a hop launch on one context (HopArgs as for
// launch_hop, the launch shape sh), its LDS bytes per block and its number of
// logical blocks. MINV: M_ee^-1 fused (Ls = 16 only).
template <class S, bool MINV>
int make_hopk(const qdwf_ctx* ctx, int prec, const HopArgs& a, const HopShape& sh, HopK* k,
              size_t* lds, int* nblocks) {
  typedef typename Store<S>::compute T;
  const Geom& g = ctx->g;
  for (int i = 0; i < 2; ++i) { k->in[i] = a.in[i]; k->out[i] = a.out[i]; k->z[i] = a.z[i]; }
  k->links = a.links ? a.links : ctx->d_links[prec];
  k->nbr = ctx->d_nbr;
  k->rs_in = a.rs_in; k->rs_out = a.rs_out; k->rs_z = a.rs_z;
  k->plane = g.n5h;
  k->Vh = g.Vh; k->Ls = g.Ls; k->nrhs = a.nrhs; k->par0 = a.par0; k->npar = a.npar;
  k->gpw = 64 / g.Ls;
  const int G = (sh.threads / 64) * k->gpw;
  k->nrb = sh.nrb;
  k->nsb = G / sh.nrb;
  k->nrblk = (a.nrhs + k->nrb - 1) / k->nrb;
  const int nsblk = (g.Vh + k->nsb - 1) / k->nsb;
  k->epi = a.epi; k->xcd = sh.xcd;
  k->c_over_b = ctx->act.c / ctx->act.b;
  k->mf = ctx->act.mf;
  k->hop_scale_b = a.hop_scale * ctx->act.b;
  k->alpha = a.alpha; k->beta = a.beta;
  k->skip = a.skip;
  k->skip_stride = a.skip_stride;
  k->cg = a.cg;
  k->cg_r = a.cg_r;
  k->cg_alpha = a.cg_alpha;
  k->cg_alpha_stride = a.cg_alpha_stride;
  k->cg_site = a.cg_site;
  k->cg_x = a.cg_x;
  k->cg_p = a.cg_p;
  if (a.cg && (a.cg > 3 || !a.epi || a.npar != 1 || !a.cg_site ||
               (a.cg >= 2 && (!a.cg_r || !a.cg_alpha)) || (a.cg == 3 && (!a.cg_x || !a.cg_p))))
    return fail(QDWF_EINVAL, "fused CG step needs a one-parity hop with epilogue and its buffers");
  k->minv = MINV;
  if (MINV) {
    if (a.epi) return fail(QDWF_EINVAL, "fused M_ee^-1 takes no epilogue term");
    const double al = ctx->act.b * (4.0 - ctx->act.M5) + 1.0;
    const double be = ctx->act.c * (4.0 - ctx->act.M5) - 1.0;
    double r = -be / al;
    for (int j = 0; j < 4; ++j) { k->rpow[j] = r; r *= r; }
    // r is now (-beta/alpha)^16 = (-beta/alpha)^Ls
    k->hop_scale_b /= al * (1.0 + ctx->act.mf * r);
  } else {
    for (int j = 0; j < 4; ++j) k->rpow[j] = 0.0;
  }
  // links, neighbour table, then (fused CG step) one double per thread
  *lds = (size_t)8 * LinkStride<T>::v * k->nsb * sizeof(T) + (size_t)8 * k->nsb * sizeof(int) +
         (a.cg ? (size_t)sh.threads * sizeof(double) : 0) + (size_t)sh.lds_pad;
  if (*lds > 64 * 1024) return fail(QDWF_EINVAL, "hop launch shape needs %zu bytes of LDS", *lds);
  *nblocks = nsblk * k->nrblk * a.npar;
  return QDWF_OK;
}

}  // namespace qdwf
