// 4D-local operators of the even-odd scheme: M_ee = alpha + beta C, its
// inverse, and their adjoints. At each 4D site they act on the Ls slices of
// one chirality at a time with a real Ls x Ls matrix (C = P- S_u + P+ S_d, so
// the upper spins 0,1 see S_d and the lower spins 2,3 see S_u). The matrices
// are built once per action on the host:
//   M_ee       upper alpha + beta S_d,  lower alpha + beta S_u
//   M_ee^dag   the transposes
//   M_ee^-1    (1/alpha) sum_k rho^k S^k / (1 + mf rho^Ls), rho = -beta/alpha,
//              with S = S_d (upper) or S_u (lower); the adjoint is its transpose.
//   (A/b) M_ee^-1 = (1 + (c/b) S) M_ee^-1, which M_pc's first stage applies.
// Kernel: the Ls lanes of a (site, rhs) group stage their 24 reals in LDS, then
// each lane forms its output slice as an Ls-term sum over the staged column.
#include <cmath>

#include "localbody.h"

namespace qdwf {

namespace {

// grid: x = site blocks, y = half index * nrhs + rhs
template <class S, int LAYOUT>
__global__ void __launch_bounds__(256) local_kernel(const S* in, S* out,
                                                    const typename Store<S>::compute* __restrict__ K,
                                                    int Vh, int Ls, long plane, long rs_half,
                                                    long rs, int nhalf) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int h = blockIdx.y % nhalf, r = blockIdx.y / nhalf;
  const long off = (long)r * rs + (long)h * rs_half;
  local_block<S, LAYOUT>(in + off, out + off, K, Vh, Ls, plane, blockIdx.x, smem);
}

}  // namespace

// Host construction of the chiral matrices of every kind: [kind][2][Ls][Ls].
std::vector<double> build_local_matrices(const qdwf_action& a) {
  const int Ls = a.Ls;
  const double al = a.b * (4.0 - a.M5) + 1.0;
  const double be = a.c * (4.0 - a.M5) - 1.0;
  std::vector<double> Su(Ls * Ls, 0.0), Sd(Ls * Ls, 0.0);
  for (int s = 0; s < Ls; ++s) {
    if (s + 1 < Ls) Su[s * Ls + s + 1] = 1.0; else Su[s * Ls] = -a.mf;
    if (s > 0) Sd[s * Ls + s - 1] = 1.0; else Sd[s * Ls + Ls - 1] = -a.mf;
  }
  std::vector<double> out((size_t)MAT_COUNT * 2 * Ls * Ls, 0.0);
  auto at = [&](int kind, int chir, int s, int t) -> double& {
    return out[(((size_t)kind * 2 + chir) * Ls + s) * Ls + t];
  };
  const double rho = -be / al;
  const double den = al * (1.0 + a.mf * std::pow(rho, Ls));
  for (int chir = 0; chir < 2; ++chir) {
    const std::vector<double>& S = chir == 0 ? Sd : Su;
    // powers of S accumulate the inverse series
    std::vector<double> P(Ls * Ls, 0.0), Q(Ls * Ls, 0.0);
    for (int s = 0; s < Ls; ++s) P[s * Ls + s] = 1.0;
    double rk = 1.0;
    std::vector<double> inv(Ls * Ls, 0.0);
    for (int k = 0; k < Ls; ++k) {
      for (int i = 0; i < Ls * Ls; ++i) inv[i] += rk * P[i] / den;
      // P <- P S
      for (int s = 0; s < Ls; ++s)
        for (int t = 0; t < Ls; ++t) {
          double acc = 0;
          for (int m = 0; m < Ls; ++m) acc += P[s * Ls + m] * S[m * Ls + t];
          Q[s * Ls + t] = acc;
        }
      P.swap(Q);
      rk *= rho;
    }
    const double cob = a.c / a.b;
    for (int s = 0; s < Ls; ++s)
      for (int t = 0; t < Ls; ++t) {
        const double m = (s == t ? al : 0.0) + be * S[s * Ls + t];
        at(MAT_MEE, chir, s, t) = m;
        at(MAT_MEE_DAG, chir, t, s) = m;
        at(MAT_MEEINV, chir, s, t) = inv[s * Ls + t];
        at(MAT_MEEINV_DAG, chir, t, s) = inv[s * Ls + t];
        // (1 + (c/b) S) M_ee^-1 on this chirality
        double am = inv[s * Ls + t];
        for (int m2 = 0; m2 < Ls; ++m2) am += cob * S[s * Ls + m2] * inv[m2 * Ls + t];
        at(MAT_AMEEINV, chir, s, t) = am;
      }
  }
  return out;
}

int launch_local(qdwf_ctx* ctx, int prec, int layout, MatKind kind, void* out, const void* in,
                 int nhalf, long rs_half, long rs, int nrhs, hipStream_t st) {
  const Geom& g = ctx->g;
  auto go = [&](auto stag) -> int {
    typedef decltype(stag) S;
    typedef typename Store<S>::compute T;
    // largest block (<= 256 threads) whose staged columns fit in 48 KB of LDS
    int threads = 256;
    while (threads > 64 &&
           ((size_t)(threads / 64) * (64 / g.Ls) * g.Ls * 24 + 2 * g.Ls * g.Ls) * sizeof(T) > 48 * 1024)
      threads /= 2;
    const int G = (threads / 64) * (64 / g.Ls);
    dim3 grid((g.Vh + G - 1) / G, nhalf * nrhs), block(threads);
    const T* K;
    if (sizeof(T) == 8) K = reinterpret_cast<const T*>(ctx->d_mat64 + (size_t)kind * 2 * g.Ls * g.Ls);
    else K = reinterpret_cast<const T*>(ctx->d_mat32 + (size_t)kind * 2 * g.Ls * g.Ls);
    const size_t lds = ((size_t)G * g.Ls * 24 + 2 * g.Ls * g.Ls) * sizeof(T);
    if (layout == QDWF_RIRI)
      hipLaunchKernelGGL((local_kernel<S, QDWF_RIRI>), grid, block, lds, st,
                         reinterpret_cast<const S*>(in), reinterpret_cast<S*>(out), K, g.Vh, g.Ls,
                         g.n5h, rs_half, rs, nhalf);
    else
      hipLaunchKernelGGL((local_kernel<S, QDWF_RRII>), grid, block, lds, st,
                         reinterpret_cast<const S*>(in), reinterpret_cast<S*>(out), K, g.Vh, g.Ls,
                         g.n5h, rs_half, rs, nhalf);
    QDWF_HIP(hipGetLastError());
    return QDWF_OK;
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
