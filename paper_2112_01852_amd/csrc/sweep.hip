// t-sweep traversal of the Domain Wall kernel: the full operator D (or
// D^dag) on both parities in one launch, Ls = 16, interleaved layout, 32- or
// 16-bit storage. The arithmetic per 5D site is the checkerboard kernel's
// (Section 4.1, 1320 flops per site in Table 3); what changes is where the
// neighbour spinors come from.
//
// The checkerboard kernel gathers all eight neighbour spinors of a 5D site
// through the vector memory path. Here a block owns one whole x-row (the Lx
// sites at fixed y, z, all 16 slices; lane = (x, s)) and walks it along t,
// one plane per step:
//   * each lane loads its own column's spinor at t+1 once: it is the +t
//     neighbour of this plane and goes into the row exchange for the next;
//   * the row's spinors at t and t-1 sit in a double-buffered LDS exchange,
//     which gives the +-x neighbours (the row is periodic in x), the -t
//     neighbour and the site's own term (a lane reads its own slot back);
//   * only the four y and z neighbours are gathered from memory, three of
//     them issued at the top of the plane;
//   * the 8 links of each site come from a doubled link field (U_mu(x) and
//     U_mu(x - mu) contiguous per site), staged in LDS one plane ahead and
//     shared by the 16 slices; links and output bypass L2 (non-temporal).
// That is five spinor loads per 5D site instead of nine. For D (not D^dag,
// 32-bit and FP16 storage) the row exchange holds chi = A psi / b rather than
// psi, so the -t, +-x and +t hops take A once per loaded column instead of
// once per neighbour; the site's own psi is then never read back: the
// 5D term (alpha + beta C) psi, divided by the hop factor, seeds the
// plane's accumulator when its column arrives, one plane ahead. The rows an XCD
// works on at one time form a compact (y, z) patch, so the y and z
// neighbours its blocks gather were loaded one plane earlier by the patch's
// other blocks and are mostly still in that XCD's L2.
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "hopcore.h"
#include "siteio.h"
#include "spin.h"

namespace qdwf {

namespace {

struct SweepK {
  const void* f;     // input field: parity-0 half, then parity-1 half
  void* o;           // output field, same layout
  const void* dl;    // doubled links [2][Vh][8][18]
  const int* idx;    // [V] internal index of each lex site
  long half, rs;     // reals per half field, reals between right-hand sides
  int Ly, Lz, Lt, Vh;
  int ntc, tl;       // t chunks per row and planes per chunk
  int ty, tz;        // (y, z) patch of rows taken in order
  int xcd;
  float cob, mf, hsb, alpha, beta;   // c/b, m_f, hop scale times b, epilogue
};

constexpr int SITE = 384;   // reals of the 16 slices of a 4D site

// Streaming accesses: the links and the output are touched once per launch,
// so they go around L2 (non-temporal), which then keeps the spinors that
// neighbouring rows read again.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <class S> __device__ inline uint4 load_nt(const S* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
// one 5D site (this lane's slice s of 4D site i) of the interleaved layout
template <class S> struct StoreNT;
template <> struct StoreNT<float> {
  __device__ static inline void run(float* f, long i, int s, const float* v) {
    f32x4* p = reinterpret_cast<f32x4*>(f + i * SITE + (long)s * 4);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const f32x4 w = {v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]};
      __builtin_nontemporal_store(w, p + c * 16);
    }
  }
};
template <class S> struct StoreNT16 {
  __device__ static inline void run(S* f, long i, int s, const float* v) {
    u32x2* p = reinterpret_cast<u32x2*>(f + i * SITE + (long)s * 4);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const u32x2 w = {pack(v[4 * c], v[4 * c + 1]), pack(v[4 * c + 2], v[4 * c + 3])};
      __builtin_nontemporal_store(w, p + c * 16);
    }
  }
  __device__ static inline unsigned pack(float a, float b) {
    const S x = Store<S>::from(a), y = Store<S>::from(b);
    unsigned short ua, ub;
    __builtin_memcpy(&ua, &x, 2);
    __builtin_memcpy(&ub, &y, 2);
    return (unsigned)ua | ((unsigned)ub << 16);
  }
};
template <> struct StoreNT<_Float16> : StoreNT16<_Float16> {};
template <> struct StoreNT<bf16> : StoreNT16<bf16> {};
constexpr int LSTR = 20;    // reals per staged link (16-byte rows)

// One hop direction D of a lane's 5D site, accumulated into acc: the
// neighbour spinor src (raw psi), for D (not D^dag) first multiplied by
// A / b = 1 + (c/b) C with the s +- 1 values from the neighbouring lanes of the
// DPP row unless PRE says src already holds A psi / b; projected to a half
// spinor, multiplied by the link at lks + D * LSTR (U_mu(x) forward,
// U_mu(x - mu)^dag backward) and reconstructed.
// refill() runs once src has been read, so a buffer may be reloaded there.
template <bool DAG, int D, bool FIRST, class Refill, bool PRE = false>
__device__ inline __attribute__((always_inline)) void dir_acc(
    const SShift<true>& sh, float cm, float cp, const float* lks, const float* src, float* acc,
    Refill refill) {
  constexpr int MU = D & 3;
  constexpr bool FWD = D < 4;
  // (1 - g) on forward hops and (1 + g) on backward ones; swapped for D^dag
  constexpr int SG = (FWD != DAG) ? -1 : +1;
  float v[24];
  if constexpr (!DAG && !PRE) {
    // chi / b = psi + (c/b) (P+ psi_{s-1} + P- psi_{s+1}), walls included
#pragma unroll
    for (int i = 0; i < 24; ++i) v[i] = src[i];
    sh.shift24i<1, 15>(cm, cp, v);
  } else {
#pragma unroll
    for (int i = 0; i < 24; ++i) v[i] = src[i];
  }
  refill();
  float h[12], uh[12], U[18];
  load_link(lks + D * LSTR, U);
  project<MU, SG>(v, h);
  su3_mul<!FWD>(U, h, uh);
  recon_acc<MU, SG, FIRST>(uh, acc);
}

// The 5D end of the full operator on the accumulated hop h (acc) of a lane:
// for D^dag first h <- A^dag h / b; then out = hop_scale b h + alpha psi +
// beta C psi (C^dag for D^dag), psi the lane's own site.
template <bool DAG>
__device__ inline __attribute__((always_inline)) void epilogue(
    const SShift<true>& sh, float cm, float cp, float hs, float al, float bm, float bp,
    const float* psi, float* acc) {
  if constexpr (DAG) {
    // A^dag h / b = h + (c/b) C^dag h: upper spins from s+1, lower from s-1
    sh.shift24i<15, 1>(cp, cm, acc);
  }
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = fmac(al, psi[i], hs * acc[i]);
  if constexpr (!DAG)
    sh.shift24<1, 15>(bm, bp, psi, acc);
  else
    sh.shift24<15, 1>(bp, bm, psi, acc);
}

// v = A psi / b = psi + (c/b) C psi for one lane (cm, cp: c/b times the wall
// factors of S_d and S_u at this slice)
__device__ inline __attribute__((always_inline)) void apply_a(
    const SShift<true>& sh, float cm, float cp, const float* psi, float* v) {
#pragma unroll
  for (int i = 0; i < 24; ++i) v[i] = psi[i];
  sh.shift24i<1, 15>(cm, cp, v);
}

// acc = (alpha psi + beta C psi) / (hop scale b): the 5D term of D in the
// units of the hop sum, so that the plane's output is (hop scale b) acc
__device__ inline __attribute__((always_inline)) void local_init(
    const SShift<true>& sh, float ial, float ibm, float ibp, const float* psi, float* acc) {
#pragma unroll
  for (int i = 0; i < 24; ++i) acc[i] = ial * psi[i];
  sh.shift24<1, 15>(ibm, ibp, psi, acc);
}

template <class S, bool DAG, int W>
__global__ void __launch_bounds__(W * 16) __attribute__((amdgpu_waves_per_eu(2, 2)))
sweep_kernel(SweepK k) {
  constexpr int NT = W * 16;
  // links of one site in 16-byte words, and words per thread per step
  constexpr int E = 16 / (int)sizeof(S);
  constexpr int CPS = 144 / E;
  constexpr int NCH = (W * CPS + NT - 1) / NT;
  __shared__ __align__(16) float X[2][W * SITE];        // the row at t (psi, or A psi / b)
  __shared__ __align__(16) float Lk[2][W * 8 * LSTR];   // the row's links at t
  __shared__ int cbrow[2][W];                            // the row's sites at t

  const int Lx = W, Ly = k.Ly, Lz = k.Lz, Lt = k.Lt;
  // logical block: right-hand side outermost, then t chunk, then rows in
  // (y, z) patches; the XCD remap gives each XCD a contiguous range
  const int B = k.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int nrow = Ly * Lz;
  const int rowi = B % nrow;
  const int rest = B / nrow;
  const int tc = rest % k.ntc;
  const int r = rest / k.ntc;
  const int psz = k.ty * k.tz;
  const int patch = rowi / psz, w = rowi - patch * psz;
  const int npy = Ly / k.ty;
  const int y = (patch % npy) * k.ty + w % k.ty;
  const int z = (patch / npy) * k.tz + w / k.ty;

  const int x = threadIdx.x >> 4, s = threadIdx.x & 15;
  const S* F = reinterpret_cast<const S*>(k.f) + (long)r * k.rs;
  S* O = reinterpret_cast<S*>(k.o) + (long)r * k.rs;
  const S* DL = reinterpret_cast<const S*>(k.dl);
  const int* idx = k.idx;

  const int yp = y + 1 == Ly ? 0 : y + 1, ym = y == 0 ? Ly - 1 : y - 1;
  const int zp = z + 1 == Lz ? 0 : z + 1, zm = z == 0 ? Lz - 1 : z - 1;
  const int xp = x + 1 == Lx ? 0 : x + 1, xm = x == 0 ? Lx - 1 : x - 1;
  const int pyz = (y + z) & 1;
  auto tmod = [&](int t) { t %= Lt; return t < 0 ? t + Lt : t; };
  auto site = [&](int xx, int yy, int zz, int t) {
    return idx[((tmod(t) * Lz + zz) * Ly + yy) * Lx + xx];
  };
  auto ld = [&](int par, int cb, float* v) {
    SiteIO<S, QDWF_RIRI>::load(F + par * k.half, cb, s, 16, 0, v);
  };
  auto store_nt = [&](S* f, int cb, const float* v) { StoreNT<S>::run(f, cb, s, v); };

  SShift<true> sh;
  sh.src_m = sh.src_p = 0;   // unused on the DPP path
  const float mf = k.mf;
  const float wm = (s == 0) ? -mf : 1.0f;    // wall factor of S_d at this slice
  const float wp = (s == 15) ? -mf : 1.0f;   // wall factor of S_u at this slice
  const float cm = k.cob * wm, cp = k.cob * wp;
  // D keeps chi = A psi / b in the row exchange (BF16 storage would spill)
  constexpr bool CHI = !DAG && !std::is_same<S, bf16>::value;
  const float ihs = 1.0f / k.hsb;
  const float ial = k.alpha * ihs, ibm = k.beta * wm * ihs, ibp = k.beta * wp * ihs;
  float acc[24];   // the plane's hop sum (with CHI: seeded one plane ahead)

  // link stage: this thread's 16-byte words of the row's doubled links
  uint4 lw[NCH];
  auto stage_load = [&](int t) {
    const int* cbr = cbrow[t & 1];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int c = threadIdx.x + j * NT;
      if (c < W * CPS) {
        const int gs = c / CPS, q = c - gs * CPS;
        const int par = (gs + pyz + t) & 1;
        const S* src = DL + ((long)par * k.Vh + cbr[gs]) * 144 + q * E;
        lw[j] = load_nt(src);   // read once per launch: keep it out of L2
      }
    }
  };
  auto stage_store = [&](int t) {
    float* dst = Lk[t & 1];
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int c = threadIdx.x + j * NT;
      if (c < W * CPS) {
        const int gs = c / CPS, q = c - gs * CPS;
        S v[E];
        __builtin_memcpy(v, &lw[j], 16);
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int e = q * E + m;   // real of the site's 144
          const int d = e / 18;
          dst[(gs * 8 + d) * LSTR + (e - d * 18)] = Store<S>::to(v[m]);
        }
      }
    }
  };

  const int t0 = tc * k.tl, tend = t0 + k.tl;
  // own column at t and t+1, and the y and z neighbours at t
  int c0 = site(x, y, z, t0), c1 = site(x, y, z, t0 + 1);
  int nyp = site(x, yp, z, t0), nym = site(x, ym, z, t0);
  int nzp = site(x, y, zp, t0), nzm = site(x, y, zm, t0);
  // the lane's slot of the row exchange: only this lane writes it, so the
  // lane may read its own column back from the previous plane's buffer
  auto put = [&](int t, const float* v) {
    float4* xs = reinterpret_cast<float4*>(X[t & 1] + x * SITE + s * 4);
#pragma unroll
    for (int c = 0; c < 6; ++c) xs[c * 16] = make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
  };
  auto get = [&](int t, int xx, float* v) {
    const float4* xs = reinterpret_cast<const float4*>(X[t & 1] + xx * SITE + s * 4);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float4 w4 = xs[c * 16];
      v[4 * c] = w4.x; v[4 * c + 1] = w4.y; v[4 * c + 2] = w4.z; v[4 * c + 3] = w4.w;
    }
  };
  {
    const int p0 = (x + pyz + t0) & 1;
    float w[24];
    ld(1 - p0, site(x, y, z, t0 - 1), w);
    // the -t neighbour of the first plane, then the first plane itself
    if constexpr (CHI) {
      float v[24];
      apply_a(sh, cm, cp, w, v);
      put(t0 - 1, v);
      ld(p0, c0, w);
      apply_a(sh, cm, cp, w, v);
      put(t0, v);
      local_init(sh, ial, ibm, ibp, w, acc);
    } else {
      put(t0 - 1, w);
      ld(p0, c0, w);
      put(t0, w);
    }
    if (s == 0) cbrow[t0 & 1][x] = c0;
    __syncthreads();
    stage_load(t0);
  }

  for (int t = t0; t < tend; ++t) {
    const int p = (x + pyz + t) & 1, q = 1 - p;
    const bool more = t + 1 < tend;
    // publish this plane's links (the row at t is already in X[t & 1])
    // and the sites of the next plane for its link stage
    stage_store(t);
    if (s == 0) cbrow[(t + 1) & 1][x] = c1;
    __syncthreads();
    // the own column at t+1: the +t neighbour, taken last in this plane, and
    // the next plane's row exchange; the y and z neighbours of the next
    // plane then read it one plane after it was loaded, while it is still in
    // this XCD's L2
    float R[24], va[24], vb[24], vc[24];
    ld(q, nyp, va);
    ld(q, nym, vb);
    ld(q, nzp, vc);
    ld(q, c1, R);
    // indices of the next plane
    const int c2 = site(x, y, z, t + 2);
    const int nyp1 = site(x, yp, z, t + 1), nym1 = site(x, ym, z, t + 1);
    const int nzp1 = site(x, y, zp, t + 1), nzm1 = site(x, y, zm, t + 1);
    if (more) stage_load(t + 1);

    const float* lks = Lk[t & 1] + x * 8 * LSTR;
    auto dir = [&](auto Dc, auto Fc, const float* src, auto refill) __attribute__((always_inline)) {
      dir_acc<DAG, decltype(Dc)::value, decltype(Fc)::value>(sh, cm, cp, lks, src, acc, refill);
    };
    // a hop from the row exchange: with CHI it holds A psi / b, and acc is
    // already seeded, so no direction starts the sum
    auto xdir = [&](auto Dc, auto Fc, const float* src, auto refill) __attribute__((always_inline)) {
      if constexpr (CHI)
        dir_acc<DAG, decltype(Dc)::value, false, decltype(refill), true>(sh, cm, cp, lks, src, acc, refill);
      else
        dir_acc<DAG, decltype(Dc)::value, decltype(Fc)::value>(sh, cm, cp, lks, src, acc, refill);
    };
    auto none = [] {};
    {
      // -t from the lane's own slot of the previous plane, which then takes
      // the next plane (no other lane reads that buffer during this plane)
      float w[24];
      get(t - 1, x, w);
      xdir(IC<7>(), std::true_type(), w, none);
    }
    {
      float w[24];
      get(t, xp, w);
      xdir(IC<0>(), std::false_type(), w, none);                             // +x
    }
    {
      float w[24];
      get(t, xm, w);
      xdir(IC<4>(), std::false_type(), w, none);                             // -x
    }
    dir(IC<1>(), std::false_type(), va, [&] { ld(q, nzm, va); });           // +y; then -z
    dir(IC<5>(), std::false_type(), vb, none);                               // -y
    dir(IC<2>(), std::false_type(), vc, none);                               // +z
    dir(IC<6>(), std::false_type(), va, none);                               // -z
    if constexpr (CHI) {
      // +t from the column just loaded, which as A psi / b becomes the next
      // plane's exchange; its psi seeds the next plane's sum
      float v[24];
      apply_a(sh, cm, cp, R, v);
      xdir(IC<3>(), std::false_type(), v, [&] { put(t + 1, v); });
#pragma unroll
      for (int i = 0; i < 24; ++i) acc[i] *= k.hsb;
      store_nt(O + p * k.half, c0, acc);
      local_init(sh, ial, ibm, ibp, R, acc);
    } else {
      dir(IC<3>(), std::false_type(), R, [&] { put(t + 1, R); });           // +t
      {
        // psi of the own site, read back from the lane's exchange slot
        float z0[24];
        get(t, x, z0);
        epilogue<DAG>(sh, cm, cp, k.hsb, k.alpha, k.beta * wm, k.beta * wp, z0, acc);
      }
      store_nt(O + p * k.half, c0, acc);
    }
    c0 = c1; c1 = c2;
    nyp = nyp1; nym = nym1; nzp = nzp1; nzm = nzm1;
  }
}

template <class S>
__global__ void dlink_kernel(const S* __restrict__ links, S* __restrict__ dl,
                             const int* __restrict__ nbr, int Vh) {
  const long total = 2L * Vh * 8;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long)gridDim.x * blockDim.x) {
    const int d = (int)(i & 7);
    const long sidx = i >> 3;
    const int cb = (int)(sidx % Vh), p = (int)(sidx / Vh);
    const int mu = d & 3;
    // forward: U_mu(x) at x; backward: U_mu(x - mu), stored at x - mu (other parity)
    const S* src = d < 4 ? links + (((long)p * 4 + mu) * Vh + cb) * 18
                         : links + (((long)(1 - p) * 4 + mu) * Vh + nbr[((long)p * 8 + d) * Vh + cb]) * 18;
    S* dst = dl + i * 18;
#pragma unroll
    for (int e = 0; e < 18; ++e) dst[e] = src[e];
  }
}

template <class S, bool DAG>
int run_sweep_w(const SweepK& k, int W, unsigned blocks, hipStream_t st) {
  switch (W) {
    case 8: hipLaunchKernelGGL((sweep_kernel<S, DAG, 8>), dim3(blocks), dim3(128), 0, st, k); break;
    case 16: hipLaunchKernelGGL((sweep_kernel<S, DAG, 16>), dim3(blocks), dim3(256), 0, st, k); break;
    case 24: hipLaunchKernelGGL((sweep_kernel<S, DAG, 24>), dim3(blocks), dim3(384), 0, st, k); break;
    case 32: hipLaunchKernelGGL((sweep_kernel<S, DAG, 32>), dim3(blocks), dim3(512), 0, st, k); break;
    default: return fail(QDWF_EINVAL, "t-sweep needs Lx in {8, 16, 24, 32}");
  }
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

int gcd(int a, int b) { while (b) { const int t = a % b; a = b; b = t; } return a; }

}  // namespace

bool sweep_geometry(const Geom& g) {
  const int Lx = g.L[0];
  return g.Ls == 16 && (Lx == 8 || Lx == 16 || Lx == 24 || Lx == 32) && g.L[3] >= 2;
}

bool sweep_eligible(const qdwf_ctx* ctx, int prec, int layout, const HopArgs& a) {
  if (!sweep_geometry(ctx->g) || layout != QDWF_RIRI) return false;
  if (prec != QDWF_F32 && prec != QDWF_F16 && prec != QDWF_BF16) return false;
  if (!ctx->d_dlinks[prec]) return false;
  if (a.npar != 2 || a.par0 != 0 || !a.epi || a.minv || a.links || a.skip || a.hop_scale == 0.0)
    return false;
  // one full field: in[p] is the other parity's half, z[p] this parity's
  const long half = ctx->g.n5h * 24;
  const size_t hb = (size_t)half * prec_bytes(prec);
  const char* f = reinterpret_cast<const char*>(a.z[0]);
  if (a.in[1] != f || a.in[0] != f + hb || a.z[1] != f + hb) return false;
  if (reinterpret_cast<const char*>(a.out[1]) != reinterpret_cast<const char*>(a.out[0]) + hb)
    return false;
  return a.rs_in == 2 * half && a.rs_out == 2 * half && a.rs_z == 2 * half;
}

int launch_sweep(qdwf_ctx* ctx, int prec, int dagger, const HopArgs& a, hipStream_t st) {
  if (!sweep_eligible(ctx, prec, QDWF_RIRI, a)) return fail(QDWF_EINVAL, "t-sweep does not apply");
  const Geom& g = ctx->g;
  const int W = g.L[0];
  SweepK k;
  k.f = a.z[0];
  k.o = a.out[0];
  k.dl = ctx->d_dlinks[prec];
  k.idx = ctx->d_idx;
  k.half = g.n5h * 24;
  k.rs = a.rs_in;
  k.Ly = g.L[1]; k.Lz = g.L[2]; k.Lt = g.L[3]; k.Vh = g.Vh;
  // rows resident at once: 8 waves per CU, 256 CUs
  const int per_cu = 32 / W >= 1 ? 32 / W : 1;
  const int resident = 256 * per_cu;
  const long nrow = (long)g.L[1] * g.L[2];
  // split t into chunks while there are too few blocks to fill the chip twice
  int ntc = 1;
  while (nrow * a.nrhs * ntc < 2L * resident && g.L[3] % (2 * ntc) == 0 && g.L[3] / (2 * ntc) >= 4)
    ntc *= 2;
  k.ntc = ntc;
  k.tl = g.L[3] / ntc;
  // an XCD's resident rows: 32 CUs x per_cu, as a (y, z) patch
  k.ty = gcd(g.L[1], per_cu >= 2 ? 16 : 8);
  k.tz = gcd(g.L[2], per_cu >= 4 ? 8 : 4);
  k.xcd = 1;
  k.cob = (float)(ctx->act.c / ctx->act.b);
  k.mf = (float)ctx->act.mf;
  k.hsb = (float)(a.hop_scale * ctx->act.b);
  k.alpha = (float)a.alpha;
  k.beta = (float)a.beta;
  const long blocks = nrow * ntc * a.nrhs;
  if (blocks > 0x7fffffffL) return fail(QDWF_EINVAL, "too many blocks for one launch");
  auto go = [&](auto tag) -> int {
    typedef decltype(tag) S;
    return dagger ? run_sweep_w<S, true>(k, W, (unsigned)blocks, st)
                  : run_sweep_w<S, false>(k, W, (unsigned)blocks, st);
  };
  switch (prec) {
    case QDWF_F32: return go(float());
    case QDWF_F16: return go(_Float16());
    case QDWF_BF16: return go(bf16());
  }
  return fail(QDWF_EINVAL, "t-sweep precision %d", prec);
}

int launch_doubled_links(qdwf_ctx* ctx, hipStream_t st) {
  const Geom& g = ctx->g;
  const long total = 2L * g.Vh * 8;
  long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  for (int p = QDWF_F32; p <= QDWF_BF16; ++p) {
    if (!ctx->d_dlinks[p]) continue;
    auto go = [&](auto tag) {
      typedef decltype(tag) S;
      hipLaunchKernelGGL(dlink_kernel<S>, dim3((unsigned)blocks), dim3(256), 0, st,
                         reinterpret_cast<const S*>(ctx->d_links[p]),
                         reinterpret_cast<S*>(ctx->d_dlinks[p]), ctx->d_nbr, g.Vh);
    };
    if (p == QDWF_F32) go(float());
    else if (p == QDWF_F16) go(_Float16());
    else go(bf16());
    QDWF_HIP(hipGetLastError());
  }
  return QDWF_OK;
}

}  // namespace qdwf
