// Body of the 4D-local operators of the even-odd scheme (M_ee, M_ee^-1 and
// their adjoints as chiral Ls x Ls matrices), shared by the launch over one
// context (local.hip) and the grouped launch over many (group.hip).
#pragma once

#include "common.h"
#include "siteio.h"

namespace qdwf {

// Block bx of out = K in on one half field: the Ls lanes of a (site, rhs)
// group stage their 24 reals in LDS, then each lane forms its output slice as
// an Ls-term sum over the staged column. K: [2][Ls][Ls] (upper chirality,
// then lower). smem: local_lds_bytes(blockDim.x, Ls, sizeof(T)) bytes.
template <class S, int LAYOUT>
__device__ inline void local_block(const S* in, S* out,
                                   const typename Store<S>::compute* __restrict__ K, int Vh,
                                   int Ls, long plane, int bx, unsigned char* smem) {
  typedef typename Store<S>::compute T;
  T* col = reinterpret_cast<T*>(smem);           // [groups][Ls][24]
  T* km = col + (blockDim.x / 64) * (64 / Ls) * Ls * 24;   // [2][Ls][Ls]
  for (int i = threadIdx.x; i < 2 * Ls * Ls; i += blockDim.x) km[i] = K[i];

  const int gpw = 64 / Ls;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane / Ls, s = lane - gl * Ls;
  const bool lane_ok = gl < gpw;
  const int gid = wave * gpw + (lane_ok ? gl : 0);
  const int G = (blockDim.x / 64) * gpw;
  const int cb = bx * G + gid;
  const bool active = lane_ok && cb < Vh;
  const int cbc = min(cb, Vh - 1);

  T v[24];
  SiteIO<S, LAYOUT>::load(in, cbc, s, Ls, plane, v);
  if (lane_ok) {
#pragma unroll
    for (int c = 0; c < 24; ++c) col[(gid * Ls + s) * 24 + c] = v[c];
  }
  __syncthreads();
  if (active) {
    T o[24];
#pragma unroll
    for (int c = 0; c < 24; ++c) o[c] = 0;
    const T* ku = km + s * Ls;              // upper chirality row s
    const T* kl = km + Ls * Ls + s * Ls;    // lower chirality row s
    const T* cg = col + gid * Ls * 24;
    for (int t = 0; t < Ls; ++t) {
      const T a = ku[t], b = kl[t];
#pragma unroll
      for (int c = 0; c < 12; ++c) o[c] += a * cg[t * 24 + c];
#pragma unroll
      for (int c = 12; c < 24; ++c) o[c] += b * cg[t * 24 + c];
    }
    SiteIO<S, LAYOUT>::store(out, cbc, s, Ls, plane, o);
  }
}

// LDS bytes of local_block for `threads` threads per block.
inline size_t local_lds_bytes(int threads, int Ls, size_t real_bytes) {
  return ((size_t)(threads / 64) * (64 / Ls) * Ls * 24 + 2 * (size_t)Ls * Ls) * real_bytes;
}

}  // namespace qdwf
