// Packed FP16 complex arithmetic for the hop on FP16 storage: one complex
// number per 32-bit word, real part in the low half, imaginary part in the
// high half -- which is how the interleaved layout stores it, so a loaded
// spinor needs no conversion before its spin projection.
//
//   * spin projection: a + c b with c in {+1, -1, +i, -i} is one
//     v_pk_add_f16, the product by c being operand selection and sign; the
//     sum of two FP16 numbers is exact before its rounding to nearest even,
//     so the projected half spinor carries one FP16 rounding (the same as
//     projecting in FP32 and storing the result as FP16);
//   * SU(3) multiply: each real output is a chain of three v_dot2 products
//     (two FP16 products, exact in FP32, added to an FP32 accumulator); the
//     link is staged in the two sign-adjusted forms its direction needs, so
//     every product is a plain dot2;
//   * reconstruction and every later step stay in FP32.
// BF16 storage uses only the SU(3) part: its half spinor is projected in
// FP32 (there are no packed BF16 adds) and rounded to BF16 for
// v_dot2_f32_bf16 against links staged the same way.
// Everything is written with vector types and builtins, so the compiler sees
// the DOT instructions and inserts the wait states their results need before
// other VALU instructions read them.
#pragma once

#include "common.h"

namespace qdwf {

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

__device__ inline half2v as_h2(uint32_t w) { return __builtin_bit_cast(half2v, w); }
__device__ inline uint32_t as_u32(half2v h) { return __builtin_bit_cast(uint32_t, h); }

__device__ inline uint32_t swap_halves(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }

// a + c b, c = (CR, CI) in {(1,0), (-1,0), (0,1), (0,-1)}: one v_pk_add_f16
template <int CR, int CI> __device__ inline uint32_t pk_cadd(uint32_t aw, uint32_t bw) {
  const half2v a = as_h2(aw), b = as_h2(bw);
  if constexpr (CR == 1) return as_u32(a + b);
  else if constexpr (CR == -1) return as_u32(a - b);
  else if constexpr (CI == 1) return as_u32(a + (half2v){-b.y, b.x});   // (a.re - b.im, a.im + b.re)
  else return as_u32(a + (half2v){b.y, -b.x});                          // (a.re + b.im, a.im - b.re)
}

// a * b + c on both halves, one FP16 rounding each (v_pk_fma_f16)
__device__ inline uint32_t pk_fma(uint32_t a, uint32_t b, uint32_t c) {
  return as_u32(__builtin_elementwise_fma(as_h2(a), as_h2(b), as_h2(c)));
}

// c + a.lo b.lo + a.hi b.hi in FP32
__device__ inline float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2(as_h2(a), as_h2(b), c, false);
}

// The same with two BF16 products (BF16 storage: the half spinor is
// projected in FP32 and rounded to BF16 for the products).
typedef __bf16 bf162v __attribute__((ext_vector_type(2)));
__device__ inline float dot2_bf16(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf162v, a),
                                         __builtin_bit_cast(bf162v, b), c, false);
}

// Two FP32 values rounded to nearest even into one BF16 pair (lo, hi).
__device__ inline uint32_t pk_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, (bf162v){(__bf16)lo, (__bf16)hi});
}

// Two FP32 values rounded to nearest even into one FP16 pair (lo, hi).
__device__ inline uint32_t pk_f16(float lo, float hi) {
  return as_u32((half2v){(_Float16)lo, (_Float16)hi});
}

__device__ inline float f16_lo(uint32_t w) { return (float)as_h2(w).x; }
__device__ inline float f16_hi(uint32_t w) { return (float)as_h2(w).y; }

// The two words of a link element (re, im) packed for the dot2 products:
//   U h (forward hops):      re = dot2((re, -im), h), im = dot2((im, re), h);
//   U^dag h (backward hops): re = dot2((re, im), h),  im = dot2((-im, re), h).
__device__ inline void link_words(uint32_t w, bool forward, uint32_t* w0, uint32_t* w1) {
  const uint32_t s = swap_halves(w);
  *w0 = forward ? (w ^ 0x80000000u) : w;
  *w1 = forward ? s : (s ^ 0x00008000u);
}

// Half spinor h = first two rows of (1 + SG g_MU) v from a packed spinor v
// (12 words [spin*3 + colour]); h: 6 words [row*3 + colour]. The same table
// as project() in spin.h.
template <int MU, int SG> __device__ inline void project_pk(const uint32_t* v, uint32_t* h) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t s0 = v[a], s1 = v[3 + a], s2 = v[6 + a], s3 = v[9 + a];
    if constexpr (MU == 0) {        // h0 = s0 + SG i s3 ; h1 = s1 + SG i s2
      h[a] = pk_cadd<0, SG>(s0, s3);
      h[3 + a] = pk_cadd<0, SG>(s1, s2);
    } else if constexpr (MU == 1) { // h0 = s0 - SG s3 ; h1 = s1 + SG s2
      h[a] = pk_cadd<-SG, 0>(s0, s3);
      h[3 + a] = pk_cadd<SG, 0>(s1, s2);
    } else if constexpr (MU == 2) { // h0 = s0 + SG i s2 ; h1 = s1 - SG i s3
      h[a] = pk_cadd<0, SG>(s0, s2);
      h[3 + a] = pk_cadd<0, -SG>(s1, s3);
    } else {                        // h0 = s0 + SG s2 ; h1 = s1 + SG s3
      h[a] = pk_cadd<SG, 0>(s0, s2);
      h[3 + a] = pk_cadd<SG, 0>(s1, s3);
    }
  }
}

// u[row][a] = sum_b M[a][b] h[row][b], M = U (DAGL = false) or U^dag, from a
// link staged as link_words (W0, W1: 9 words each, row-major [a][b]); u in
// FP32 as (re, im) pairs, the layout su3_mul writes. BF: the words hold BF16
// pairs (the sign adjustments of link_words are the same bits).
template <bool DAGL, bool BF = false>
__device__ inline void su3_mul_pk(const uint32_t* W0, const uint32_t* W1, const uint32_t* h,
                                  float* u) {
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const uint32_t* hh = h + r * 3;
      float re = 0.0f, im = 0.0f;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int e = DAGL ? b * 3 + a : a * 3 + b;
        if constexpr (BF) {
          re = dot2_bf16(W0[e], hh[b], re);
          im = dot2_bf16(W1[e], hh[b], im);
        } else {
          re = dot2(W0[e], hh[b], re);
          im = dot2(W1[e], hh[b], im);
        }
      }
      u[(r * 3 + a) * 2] = re;
      u[(r * 3 + a) * 2 + 1] = im;
    }
}

}  // namespace qdwf
