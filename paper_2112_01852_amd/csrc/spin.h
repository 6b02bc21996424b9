// Spin and colour algebra of the 4D hop, shared by the domain-wall and the
// Wilson kernels: half-spinor projection (1 +- gamma_mu), SU(3) multiply of a
// half spinor, reconstruction, and link loads from global memory.
// Gamma matrices: chiral (DeGrand-Rossi) basis, gamma_5 = diag(1, 1, -1, -1).
#pragma once

#include "common.h"

namespace qdwf {

// ----------------------------------------------- spin projection algebra
// The constants below are compile-time, and every case is written out so that
// no multiply by 0 or +-1 and no add of 0 reaches the instruction stream (IEEE
// rules forbid the compiler from dropping those itself).
template <class T> __device__ inline T fmac(T a, T b, T c);
template <> __device__ inline float fmac<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ inline double fmac<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// o = a + c b with c in {+1, -1, +i, -i} given as (CR, CI)
template <int CR, int CI, class T>
__device__ inline void cadd(const T* a, const T* b, T* o) {
  if constexpr (CR == 1) { o[0] = a[0] + b[0]; o[1] = a[1] + b[1]; }
  else if constexpr (CR == -1) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; }
  else if constexpr (CI == 1) { o[0] = a[0] - b[1]; o[1] = a[1] + b[0]; }
  else { o[0] = a[0] + b[1]; o[1] = a[1] - b[0]; }
}
// o = c b
template <int CR, int CI, class T>
__device__ inline void cset(const T* b, T* o) {
  if constexpr (CR == 1) { o[0] = b[0]; o[1] = b[1]; }
  else if constexpr (CR == -1) { o[0] = -b[0]; o[1] = -b[1]; }
  else if constexpr (CI == 1) { o[0] = -b[1]; o[1] = b[0]; }
  else { o[0] = b[1]; o[1] = -b[0]; }
}

// Half spinor h = first two rows of (1 + SG g_MU) v, h[(hs*3 + colour)*2 + re/im].
template <int MU, int SG, class T>
__device__ inline void project(const T* v, T* h) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T* s0 = v + (0 * 3 + a) * 2;
    const T* s1 = v + (1 * 3 + a) * 2;
    const T* s2 = v + (2 * 3 + a) * 2;
    const T* s3 = v + (3 * 3 + a) * 2;
    T* h0 = h + (0 * 3 + a) * 2;
    T* h1 = h + (1 * 3 + a) * 2;
    if constexpr (MU == 0) {        // h0 = s0 + SG i s3 ; h1 = s1 + SG i s2
      cadd<0, SG>(s0, s3, h0);
      cadd<0, SG>(s1, s2, h1);
    } else if constexpr (MU == 1) { // h0 = s0 - SG s3 ; h1 = s1 + SG s2
      cadd<-SG, 0>(s0, s3, h0);
      cadd<SG, 0>(s1, s2, h1);
    } else if constexpr (MU == 2) { // h0 = s0 + SG i s2 ; h1 = s1 - SG i s3
      cadd<0, SG>(s0, s2, h0);
      cadd<0, -SG>(s1, s3, h1);
    } else {                        // h0 = s0 + SG s2 ; h1 = s1 + SG s3
      cadd<SG, 0>(s0, s2, h0);
      cadd<SG, 0>(s1, s3, h1);
    }
  }
}

// acc (+)= (1 + SG g_MU) psi rebuilt from the multiplied half spinor u:
// rows 0,1 are u0,u1; rows 2,3 are fixed multiples of u0 or u1.
template <int MU, int SG, bool FIRST, class T>
__device__ inline void recon_acc(const T* u, T* acc) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T* u0 = u + (0 * 3 + a) * 2;
    const T* u1 = u + (1 * 3 + a) * 2;
    T* r0 = acc + (0 * 3 + a) * 2;
    T* r1 = acc + (1 * 3 + a) * 2;
    T* r2 = acc + (2 * 3 + a) * 2;
    T* r3 = acc + (3 * 3 + a) * 2;
    // r2 = c2 u_j2, r3 = c3 u_j3 with (c, j) from the gamma matrix
    constexpr int C2R = MU == 1 ? SG : (MU == 3 ? SG : 0);
    constexpr int C2I = MU == 0 ? -SG : (MU == 2 ? -SG : 0);
    constexpr int C3R = MU == 1 ? -SG : (MU == 3 ? SG : 0);
    constexpr int C3I = MU == 0 ? -SG : (MU == 2 ? SG : 0);
    const T* j2 = (MU == 0 || MU == 1) ? u1 : u0;
    const T* j3 = (MU == 0 || MU == 1) ? u0 : u1;
    if constexpr (FIRST) {
      r0[0] = u0[0]; r0[1] = u0[1];
      r1[0] = u1[0]; r1[1] = u1[1];
      cset<C2R, C2I>(j2, r2);
      cset<C3R, C3I>(j3, r3);
    } else {
      r0[0] += u0[0]; r0[1] += u0[1];
      r1[0] += u1[0]; r1[1] += u1[1];
      cadd<C2R, C2I>(r2, j2, r2);
      cadd<C3R, C3I>(r3, j3, r3);
    }
  }
}

// u[hs][a] = sum_b M[a][b] h[hs][b] with M = U (DAGL = false) or U^dag:
// one multiply and five fused multiply-adds per real output.
template <bool DAGL, class T>
__device__ inline void su3_mul(const T* U, const T* h, T* u) {
#pragma unroll
  for (int hs = 0; hs < 2; ++hs)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* hh = h + hs * 6;
      T re, im;
      if constexpr (!DAGL) {
        const T* m = U + a * 6;   // row a: U[a][b] at m + 2b
        re = m[0] * hh[0];
        im = m[0] * hh[1];
        re = fmac(-m[1], hh[1], re);
        im = fmac(m[1], hh[0], im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
          re = fmac(m[2 * b], hh[2 * b], re);
          im = fmac(m[2 * b], hh[2 * b + 1], im);
          re = fmac(-m[2 * b + 1], hh[2 * b + 1], re);
          im = fmac(m[2 * b + 1], hh[2 * b], im);
        }
      } else {
        // conj(U[b][a]) at column a of row b: U + b*6 + 2a
        const T* m = U + 2 * a;
        re = m[0] * hh[0];
        im = m[0] * hh[1];
        re = fmac(m[1], hh[1], re);
        im = fmac(-m[1], hh[0], im);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
          const T* mb = m + 6 * b;
          re = fmac(mb[0], hh[2 * b], re);
          im = fmac(mb[0], hh[2 * b + 1], im);
          re = fmac(mb[1], hh[2 * b + 1], re);
          im = fmac(-mb[1], hh[2 * b], im);
        }
      }
      u[(hs * 3 + a) * 2] = re;
      u[(hs * 3 + a) * 2 + 1] = im;
    }
}

// A link (3x3 complex, 18 reals) from global memory: 8-byte loads for the
// 32- and 64-bit types (a link starts on an 8-byte boundary), 4-byte loads for
// the 16-bit types.
template <class S> struct LinkIO {
  typedef typename Store<S>::compute T;
  __device__ static inline void load(const S* __restrict__ p, T* U) {
    if constexpr (sizeof(S) == 8) {
      const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double2 w = q[k];
        U[2 * k] = (T)w.x; U[2 * k + 1] = (T)w.y;
      }
    } else if constexpr (sizeof(S) == 4) {
      const float2* q = reinterpret_cast<const float2*>(p);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float2 w = q[k];
        U[2 * k] = (T)w.x; U[2 * k + 1] = (T)w.y;
      }
    } else {
      const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const uint32_t w = q[k];
        S a, b;
        __builtin_memcpy(&a, &w, 2);
        const uint32_t hi = w >> 16;
        __builtin_memcpy(&b, &hi, 2);
        U[2 * k] = Store<S>::to(a); U[2 * k + 1] = Store<S>::to(b);
      }
    }
  }
};

template <int N> struct IC { static constexpr int value = N; };

}  // namespace qdwf
