// Pieces of the Domain Wall kernel shared by its two traversals (one lane
// per 5D site in checkerboard order, and the t-sweep of whole x-rows): the
// XCD-aware block renumbering, link loads into registers, and the s +- 1
// exchange between the slices of a site held by neighbouring lanes.
#pragma once

#include "common.h"
#include "spin.h"

namespace qdwf {

__device__ inline int xcd_remap(int bid, int nb) {
  // hardware hands block i to XCD i % 8; give XCD x a contiguous range instead
  const int per = nb >> 3, rem = nb & 7;
  const int x = bid & 7, k = bid >> 3;
  return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Link staging stride in LDS (reals per link): 16-byte aligned rows.
template <class T> struct LinkStride { static constexpr int v = 20; };
template <> struct LinkStride<double> { static constexpr int v = 18; };

template <class T>
__device__ inline void load_link(const T* __restrict__ p, T* U) {
  if constexpr (sizeof(T) == 4) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 w = q[k];
      U[4 * k] = w.x; U[4 * k + 1] = w.y; U[4 * k + 2] = w.z; U[4 * k + 3] = w.w;
    }
    const float2 w = *reinterpret_cast<const float2*>(p + 16);
    U[16] = w.x; U[17] = w.y;
  } else {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double2 w = q[k];
      U[2 * k] = w.x; U[2 * k + 1] = w.y;
    }
  }
}


// s +- 1 exchange inside a group of Ls lanes. fm(c, x, a) = a + c x(s-1) and
// fp(c, x, a) = a + c x(s+1), cyclically in s (the walls are handled by the
// caller's coefficients). Generic Ls uses cross-lane permutes.
template <bool DPP16> struct SShift {
  int src_m, src_p;
  template <class T> __device__ inline T fm(T c, T x, T a) const { return fmac(c, (T)__shfl(x, src_m, 64), a); }
  template <class T> __device__ inline T fp(T c, T x, T a) const { return fmac(c, (T)__shfl(x, src_p, 64), a); }
};

// Ls = 16: a group is one DPP row and the exchange is a row rotate. In FP32
// the rotate is the source modifier of the FMA itself (one instruction); the
// s_nop covers the two wait states a DPP read needs after a VALU write of the
// same register, which the compiler does not track through inline assembly.
// FP64 has no row rotate on 64-bit operands, so each half is moved first.
template <int R> __device__ inline int dpp_ror(int v) {
  return __builtin_amdgcn_mov_dpp(v, 0x120 + R, 0xF, 0xF, false);
}
// v_fmac_f32 with its first source read through a DPP row rotate by R lanes
#define QDWF_FMAC_ROR(R)                                                              \
  asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 row_ror:" #R " row_mask:0xf bank_mask:0xf" \
      : "+v"(a) : "v"(x), "v"(c))
// six of them, a[j] += c x[j](lane - R), after one s_nop
#define QDWF_DPP_ROR(R, D, X) "\n\tv_fmac_f32_dpp %" #D ", %" #X ", %12 row_ror:" #R " row_mask:0xf bank_mask:0xf"
#define QDWF_FMAC_ROR6(R)                                                             \
  asm("s_nop 1" QDWF_DPP_ROR(R, 0, 6) QDWF_DPP_ROR(R, 1, 7) QDWF_DPP_ROR(R, 2, 8)      \
      QDWF_DPP_ROR(R, 3, 9) QDWF_DPP_ROR(R, 4, 10) QDWF_DPP_ROR(R, 5, 11)               \
      : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5])          \
      : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(x[4]), "v"(x[5]), "v"(c))
// in place: a[j] += c a[j](lane - R), each FMA's DPP source its own register
#define QDWF_DPP_ROR_IP(R, D) "\n\tv_fmac_f32_dpp %" #D ", %" #D ", %6 row_ror:" #R " row_mask:0xf bank_mask:0xf"
#define QDWF_FMAC_ROR6_IP(R)                                                          \
  asm("s_nop 1" QDWF_DPP_ROR_IP(R, 0) QDWF_DPP_ROR_IP(R, 1) QDWF_DPP_ROR_IP(R, 2)      \
      QDWF_DPP_ROR_IP(R, 3) QDWF_DPP_ROR_IP(R, 4) QDWF_DPP_ROR_IP(R, 5)                 \
      : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5])          \
      : "v"(c))
template <> struct SShift<true> {
  int src_m, src_p;
  // a + c x(lane - R), R = 1..15, within the 16-lane row
  template <int R> __device__ inline float fr(float c, float x, float a) const {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 12 || R == 14 || R == 15,
                  "rotation not instantiated");
    if constexpr (R == 1) QDWF_FMAC_ROR(1);
    else if constexpr (R == 2) QDWF_FMAC_ROR(2);
    else if constexpr (R == 4) QDWF_FMAC_ROR(4);
    else if constexpr (R == 8) QDWF_FMAC_ROR(8);
    else if constexpr (R == 12) QDWF_FMAC_ROR(12);
    else if constexpr (R == 14) QDWF_FMAC_ROR(14);
    else QDWF_FMAC_ROR(15);
    return a;
  }
  template <int R> __device__ inline double fr(double c, double x, double a) const {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_ror<R>((int)b), hi = dpp_ror<R>((int)(b >> 32));
    return fmac(c, __longlong_as_double(((long long)hi << 32) | (unsigned int)lo), a);
  }
  template <class T> __device__ inline T fm(T c, T x, T a) const { return fr<1>(c, x, a); }
  template <class T> __device__ inline T fp(T c, T x, T a) const { return fr<15>(c, x, a); }
  // v[0..11] += cu x[0..11](lane - RU) and v[12..23] += cl x[12..23](lane -
  // RL) for one 24-real spinor (RU, RL = 1: from s-1, 15: from s+1): four
  // groups of six DPP FMAs, each behind a single pair of wait states. Within
  // a group the six sources are distinct registers that none of the six FMAs
  // writes (each is a different value live at the group's start, and an
  // output can share a register only with its own input), so no FMA reads a
  // register the group has just written.
  template <int RU, int RL>
  __device__ inline void shift24(float cu, float cl, const float* x, float* v) const {
    fr6<RU>(cu, x, v);
    fr6<RU>(cu, x + 6, v + 6);
    fr6<RL>(cl, x + 12, v + 12);
    fr6<RL>(cl, x + 18, v + 18);
  }
  // the same in place, v += c v(shifted): no source copies
  template <int RU, int RL> __device__ inline void shift24i(float cu, float cl, float* v) const {
    fr6i<RU>(cu, v);
    fr6i<RU>(cu, v + 6);
    fr6i<RL>(cl, v + 12);
    fr6i<RL>(cl, v + 18);
  }
  template <int R> __device__ inline void fr6i(float c, float* a) const {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 12 || R == 14 || R == 15,
                  "rotation not instantiated");
    if constexpr (R == 1) QDWF_FMAC_ROR6_IP(1);
    else if constexpr (R == 2) QDWF_FMAC_ROR6_IP(2);
    else if constexpr (R == 4) QDWF_FMAC_ROR6_IP(4);
    else if constexpr (R == 8) QDWF_FMAC_ROR6_IP(8);
    else if constexpr (R == 12) QDWF_FMAC_ROR6_IP(12);
    else if constexpr (R == 14) QDWF_FMAC_ROR6_IP(14);
    else QDWF_FMAC_ROR6_IP(15);
  }
  template <int R> __device__ inline void fr6(float c, const float* x, float* a) const {
    static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 12 || R == 14 || R == 15,
                  "rotation not instantiated");
    if constexpr (R == 1) QDWF_FMAC_ROR6(1);
    else if constexpr (R == 2) QDWF_FMAC_ROR6(2);
    else if constexpr (R == 4) QDWF_FMAC_ROR6(4);
    else if constexpr (R == 8) QDWF_FMAC_ROR6(8);
    else if constexpr (R == 12) QDWF_FMAC_ROR6(12);
    else if constexpr (R == 14) QDWF_FMAC_ROR6(14);
    else QDWF_FMAC_ROR6(15);
  }
};

// v[0..11] += cu x[0..11](s - RU) and v[12..23] += cu x[12..23](s - RL), s
// cyclic over the Ls slices (R = 1: from s - 1, R = Ls - 1: from s + 1). FP32
// on the DPP path goes six FMAs to a wait-state pair (SShift<true>::shift24);
// FP64 and the permute path (which knows only s -+ 1) go element by element.
template <int RU, int RL, bool DPP16, class T>
__device__ inline void shift_s(const SShift<DPP16>& sh, T cu, T cl, const T* x, T* v) {
  if constexpr (DPP16 && sizeof(T) == 4) {
    sh.template shift24<RU, RL>(cu, cl, x, v);
  } else if constexpr (DPP16) {
#pragma unroll
    for (int i = 0; i < 12; ++i) v[i] = sh.template fr<RU>(cu, x[i], v[i]);
#pragma unroll
    for (int i = 12; i < 24; ++i) v[i] = sh.template fr<RL>(cl, x[i], v[i]);
  } else {
    static_assert((RU == 1 && RL == 15) || (RU == 15 && RL == 1), "permute path shifts by one slice");
#pragma unroll
    for (int i = 0; i < 12; ++i) v[i] = RU == 1 ? sh.fm(cu, x[i], v[i]) : sh.fp(cu, x[i], v[i]);
#pragma unroll
    for (int i = 12; i < 24; ++i) v[i] = RL == 1 ? sh.fm(cl, x[i], v[i]) : sh.fp(cl, x[i], v[i]);
  }
}
#undef QDWF_FMAC_ROR
#undef QDWF_FMAC_ROR6
#undef QDWF_FMAC_ROR6_IP

}  // namespace qdwf
