// Spinor storage inside a half field (one parity) and the per-lane loads and
// stores of one 5D site. In registers the 24 reals of a site are kept in the
// order v[(spin*3 + colour)*2 + re/im].
//
//   RIRI  interleaved complex. The Ls slices of 4D site i form one block of
//         Ls*24 reals, cut into 6 chunks of 4 consecutive reals (two complex
//         numbers) and stored chunk-major, then slice:
//             offset(i, s, c) = i*Ls*24 + (c/4)*Ls*4 + s*4 + c%4.
//         The lanes holding the slices of one site read one chunk each from
//         a contiguous run of Ls chunks per load, so a wavefront's gather of
//         a neighbour touches the fewest cache lines. The element order is
//         the same in every precision, which lets the solver convert
//         between precisions element by element.
//         With Ls = 1 (4D fields) the same blocking runs over 16 consecutive
//         sites instead: site i is slice i % 16 of block i / 16, so that the
//         lanes of consecutive sites read contiguous runs (V/2 must then be a
//         multiple of 16).
//   RRII  split planes: 24 planes of n5h = (V/2)*Ls reals, plane
//         (c & 1)*12 + c/2 ([re/im][spin][colour]), index i*Ls + s.
//
// Real and imaginary part of a complex number stay adjacent in RIRI, which
// the complex reductions rely on.
#pragma once

#include "common.h"

namespace qdwf {

// Ls = 1: 16 consecutive sites play the role of the slices of a block.
__host__ __device__ inline void riri_block(long& i, int& s, int& Ls) {
  if (Ls == 1) {
    s = (int)(i & 15);
    i >>= 4;
    Ls = 16;
  }
}

__host__ __device__ inline long riri_offset(long i, int s, int c, int Ls) {
  riri_block(i, s, Ls);
  return i * Ls * 24 + (long)(c >> 2) * Ls * 4 + (long)s * 4 + (c & 3);
}

__host__ __device__ inline long rrii_offset(long i, int s, int c, int Ls, long plane) {
  return (long)((c & 1) * 12 + (c >> 1)) * plane + i * Ls + s;
}

template <class S, int LAYOUT> struct SiteIO;

template <class S> struct SiteIO<S, QDWF_RRII> {
  typedef typename Store<S>::compute T;
  __device__ static inline void load(const S* __restrict__ f, long i, int s, int Ls, long plane,
                                     T* v) {
    const long j = i * Ls + s;
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) {
      v[2 * sc] = Store<S>::to(f[(long)sc * plane + j]);
      v[2 * sc + 1] = Store<S>::to(f[(long)(12 + sc) * plane + j]);
    }
  }
  __device__ static inline void store(S* __restrict__ f, long i, int s, int Ls, long plane,
                                      const T* v) {
    const long j = i * Ls + s;
#pragma unroll
    for (int sc = 0; sc < 12; ++sc) {
      f[(long)sc * plane + j] = Store<S>::from(v[2 * sc]);
      f[(long)(12 + sc) * plane + j] = Store<S>::from(v[2 * sc + 1]);
    }
  }
};

template <> struct SiteIO<double, QDWF_RIRI> {
  __device__ static inline void load(const double* __restrict__ f, long i, int s, int Ls, long,
                                     double* v) {
    riri_block(i, s, Ls);
    const double2* p = reinterpret_cast<const double2*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double2 q0 = p[2 * k * Ls], q1 = p[2 * k * Ls + 1];
      v[4 * k] = q0.x;
      v[4 * k + 1] = q0.y;
      v[4 * k + 2] = q1.x;
      v[4 * k + 3] = q1.y;
    }
  }
  __device__ static inline void store(double* __restrict__ f, long i, int s, int Ls, long,
                                      const double* v) {
    riri_block(i, s, Ls);
    double2* p = reinterpret_cast<double2*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      p[2 * k * Ls] = make_double2(v[4 * k], v[4 * k + 1]);
      p[2 * k * Ls + 1] = make_double2(v[4 * k + 2], v[4 * k + 3]);
    }
  }
};

template <> struct SiteIO<float, QDWF_RIRI> {
  __device__ static inline void load(const float* __restrict__ f, long i, int s, int Ls, long,
                                     float* v) {
    riri_block(i, s, Ls);
    const float4* p = reinterpret_cast<const float4*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float4 q = p[k * Ls];
      v[4 * k] = q.x;
      v[4 * k + 1] = q.y;
      v[4 * k + 2] = q.z;
      v[4 * k + 3] = q.w;
    }
  }
  __device__ static inline void store(float* __restrict__ f, long i, int s, int Ls, long,
                                      const float* v) {
    riri_block(i, s, Ls);
    float4* p = reinterpret_cast<float4*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      p[k * Ls] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
  }
};

// 16-bit storage: a chunk of 4 reals is one 8-byte word.
template <class S> struct SiteIO16 {
  __device__ static inline void load(const S* __restrict__ f, long i, int s, int Ls, long,
                                     float* v) {
    riri_block(i, s, Ls);
    const uint2* p = reinterpret_cast<const uint2*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint2 q = p[k * Ls];
      v[4 * k] = Store<S>::to(bits((uint16_t)(q.x & 0xffffu)));
      v[4 * k + 1] = Store<S>::to(bits((uint16_t)(q.x >> 16)));
      v[4 * k + 2] = Store<S>::to(bits((uint16_t)(q.y & 0xffffu)));
      v[4 * k + 3] = Store<S>::to(bits((uint16_t)(q.y >> 16)));
    }
  }
  __device__ static inline void store(S* __restrict__ f, long i, int s, int Ls, long,
                                      const float* v) {
    riri_block(i, s, Ls);
    uint2* p = reinterpret_cast<uint2*>(f + i * Ls * 24 + (long)s * 4);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const uint32_t w0 = (uint32_t)raw(Store<S>::from(v[4 * k])) |
                          ((uint32_t)raw(Store<S>::from(v[4 * k + 1])) << 16);
      const uint32_t w1 = (uint32_t)raw(Store<S>::from(v[4 * k + 2])) |
                          ((uint32_t)raw(Store<S>::from(v[4 * k + 3])) << 16);
      p[k * Ls] = make_uint2(w0, w1);
    }
  }
  __device__ static inline S bits(uint16_t u);
  __device__ static inline uint16_t raw(_Float16 h) { return __builtin_bit_cast(uint16_t, h); }
  __device__ static inline uint16_t raw(bf16 h) { return h.u; }
};
template <> __device__ inline _Float16 SiteIO16<_Float16>::bits(uint16_t u) {
  return __builtin_bit_cast(_Float16, u);
}
template <> __device__ inline bf16 SiteIO16<bf16>::bits(uint16_t u) {
  bf16 r;
  r.u = u;
  return r;
}
template <> struct SiteIO<_Float16, QDWF_RIRI> : SiteIO16<_Float16> {};
template <> struct SiteIO<bf16, QDWF_RIRI> : SiteIO16<bf16> {};

}  // namespace qdwf
