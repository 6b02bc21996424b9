// Bodies of the CG vector kernels (reductions, alpha/beta, the direction and
// x passes of the fused iteration, the reliable-update steps), shared by the launches over one
// context's right-hand sides (solver.hip) and the grouped launches over many
// requests (group.hip). Each body does the work of one block `bx` of `NB`
// for right-hand side `q` (the per-right-hand-side scalar steps take only q);
// `sh` is RT doubles of LDS. A right-hand side's result depends only on its
// own data, n and NB, never on what else a launch covers, so batched,
// grouped and lone solves of it are bitwise equal.
#pragma once

#include <initializer_list>

#include "cgtypes.h"
#include "common.h"
#include "solver.h"

namespace qdwf {

constexpr int RT = 256;   // threads of reduction / BLAS kernels

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <class S> __device__ inline double rd(const S* p, long i) {
  return (double)Store<S>::to(p[i]);
}

// Work split of the vectorised BLAS kernels: block b takes a contiguous range
// of tiles of 512 reals (one stream per block through memory), its wavefronts
// taking the tiles in turn, and in tile t lane l owns the reals
// t*512 + j*64*E + l*E + e (j < 8/E, e < E), E = 16 bytes over the widest
// storage type of the kernel's fields. Every load or store of E reals is then
// one piece of a contiguous run across the wavefront.
constexpr int TILE = 512;

template <int BYTES> struct Word;
template <> struct Word<16> { typedef uint4 t; };
template <> struct Word<8> { typedef uint2 t; };
template <> struct Word<4> { typedef uint32_t t; };

// E consecutive reals of storage type S <-> compute values (one aligned word).
template <class S, int E> struct Chunk {
  typedef typename Word<E * (int)sizeof(S)>::t W;
  template <class T> __device__ static inline void ld(const S* __restrict__ p, T* v) {
    const W w = *reinterpret_cast<const W*>(p);
    S e[E];
    __builtin_memcpy(e, &w, sizeof(e));
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = (T)Store<S>::to(e[k]);
  }
  template <class T> __device__ static inline void st(S* __restrict__ p, const T* v) {
    S e[E];
#pragma unroll
    for (int k = 0; k < E; ++k) e[k] = Store<S>::from((typename Store<S>::compute)v[k]);
    W w;
    __builtin_memcpy(&w, e, sizeof(e));
    *reinterpret_cast<W*>(p) = w;
  }
};

template <class A, class B, class C = A>
struct ChunkWidth {
  static constexpr int maxb = sizeof(A) > sizeof(B) ? (sizeof(A) > sizeof(C) ? sizeof(A) : sizeof(C))
                                                     : (sizeof(B) > sizeof(C) ? sizeof(B) : sizeof(C));
  static constexpr int e = 16 / maxb;
};

// Whether arrays of storage type S at these addresses, with right-hand-side
// stride rs reals, can be walked in 16-byte words.
template <class S> inline bool vec_ok(long rs, std::initializer_list<const void*> ptrs) {
  if (((rs * (long)sizeof(S)) & 15) != 0) return false;
  for (const void* q : ptrs)
    if (reinterpret_cast<uintptr_t>(q) & 15) return false;
  return true;
}

__device__ inline double part_sum(const double* part, int NB, int r, double* sh) {
  double acc = 0;
  for (int i = threadIdx.x; i < NB; i += RT) acc += part[(long)r * NB + i];
  return block_sum(acc, sh);
}

// part[r*NB + blk] = sum over this block's share of a_r . b_r (all reals);
// vec: both fields can be read in aligned words (see TILE).
template <class SA, class SB>
__device__ inline void k_dot_body(const SA* __restrict__ a, const SB* __restrict__ b,
                                            long n, long rsa, long rsb, double* __restrict__ part,
                                            int vec,
    int bx, int NB, int q, double* sh) {
  const int r = q;
  const SA* ar = a + (long)r * rsa;
  const SB* br = b + (long)r * rsb;
  double acc = 0;
  constexpr int E = ChunkWidth<SA, SB>::e;
  const long nt = vec ? n / TILE : 0;
  const int lane = threadIdx.x & 63;
  const long t1 = nt * (bx + 1) / NB;   // this block's contiguous range of tiles
  for (long t = nt * bx / NB + (threadIdx.x >> 6); t < t1; t += RT / 64) {
#pragma unroll
    for (int j = 0; j < 8 / E; ++j) {
      const long i = t * TILE + j * 64 * E + lane * E;
      double x[E], y[E];
      Chunk<SA, E>::ld(ar + i, x);
      Chunk<SB, E>::ld(br + i, y);
#pragma unroll
      for (int k = 0; k < E; ++k) acc += x[k] * y[k];
    }
  }
  for (long i = TILE * nt + (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT)
    acc += rd(ar, i) * rd(br, i);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)r * NB + bx] = t;
}

// alpha = rr / <p, Ap>, <p, Ap> = |M_pc p|^2 from the partials; j >= 0:
// also kept as alpha_hist[j] (iteration j of a group of qdwf_solve)
__device__ inline void k_alpha_body(const double* __restrict__ part, int NB,
                                              RhsState* __restrict__ st,
    int q, double* sh, int j = -1) {
  const double pAp = part_sum(part, NB, q, sh);
  if (threadIdx.x) return;
  RhsState& s = st[q];
  s.fresh = 0;
  if (s.status != ST_RUN) return;
  s.pAp = pAp;
  if (!(pAp > 0.0) || !isfinite(pAp)) {
    s.status = ST_BREAKDOWN;
    s.alpha = 0.0;
    return;
  }
  s.alpha = s.rr / pAp;
  if (j >= 0) s.alpha_hist[j] = s.alpha;
}

// beta = rr_new / rr ; decide whether a reliable update is due
__device__ inline void k_beta_body(const double* __restrict__ part, int NB,
                                             RhsState* __restrict__ st, double delta2,
    int q, double* sh, int j = -1) {
  const double rr_new = part_sum(part, NB, q, sh);
  if (threadIdx.x) return;
  RhsState& s = st[q];
  s.xstep = s.status == ST_RUN;
  if (j >= 0) s.xmask = (j == 0 ? 0 : s.xmask) | (s.xstep << j);
  if (s.status != ST_RUN) return;
  s.iters += 1;
  if (!isfinite(rr_new)) {
    s.status = ST_NAN;
    return;
  }
  s.rr_prev = s.rr;
  s.rr = rr_new;
  s.beta = rr_new / s.rr_prev;
  if (rr_new <= s.thresh || rr_new < delta2 * s.rr_ru) s.status = ST_UPDATE;
  if (s.max_iter > 0 && s.iters >= s.max_iter) {
    // out of iterations: one more reliable update reports the true residual
    s.status = ST_UPDATE;
    s.final = 1;
  }
}

// qdwf_solve runs its iterations in groups of up to kGroupSlots and updates
// x once per group: iteration j of a group reads its search direction from
// slot j (slot stride ps reals) and writes the next one to slot j + 1; the
// last adds every step of the group to x and writes the next direction to
// slot 0, where the next group (and a reliable update) starts.
// Iteration j < last: slot j+1 = r + beta slot j while the rhs keeps running
// (one that pauses here keeps its direction in slot j). With ps = 0 and
// j = 0 it is p = r + beta p in place: the serving pool's p pass, whose x
// takes each iteration's step in the last hop of M_pc^dag.
template <class SR, class SP>
__device__ inline void k_grp_p_body(const SR* __restrict__ r, SP* __restrict__ p0, long ps, int j,
                                    long n, long rs, const RhsState* __restrict__ st, int vec,
    int bx, int NB, int q) {
  typedef typename Store<SR>::compute T;
  const RhsState& s = st[q];
  if (s.status != ST_RUN) return;
  const T be = (T)s.beta;
  const SR* rr = r + (long)q * rs;
  const SP* ar = p0 + (long)j * ps + (long)q * rs;
  SP* br = p0 + (long)(j + 1) * ps + (long)q * rs;
  constexpr int E = ChunkWidth<SR, SP>::e;
  const long nt = vec ? n / TILE : 0;
  const int lane = threadIdx.x & 63;
  const long t1 = nt * (bx + 1) / NB;
  for (long t = nt * bx / NB + (threadIdx.x >> 6); t < t1; t += RT / 64) {
#pragma unroll
    for (int jj = 0; jj < 8 / E; ++jj) {
      const long i = t * TILE + jj * 64 * E + lane * E;
      T rv[E], pv[E];
      Chunk<SR, E>::ld(rr + i, rv);
      Chunk<SP, E>::ld(ar + i, pv);
#pragma unroll
      for (int k = 0; k < E; ++k) pv[k] = rv[k] + be * pv[k];
      Chunk<SP, E>::st(br + i, pv);
    }
  }
  for (long i = TILE * nt + (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT)
    br[i] = Store<SP>::from((T)Store<SR>::to(rr[i]) + be * (T)Store<SP>::to(ar[i]));
}

// Last iteration of a group of len: x += alpha_hist[i] slot i for every
// iteration i that took its step, in order (the rounding of one update per
// iteration); then slot 0 = r + beta slot len-1 while the rhs keeps running,
// or slot 0 = slot m if it paused after its last step m > 0.
template <class SX, class SR, class SP>
__device__ inline void k_grp_last_body(SX* __restrict__ x, const SR* __restrict__ r,
                                       SP* __restrict__ p0, long ps, int len, long n, long rs,
                                       const RhsState* __restrict__ st, int vec,
    int bx, int NB, int q) {
  typedef typename Store<SR>::compute T;
  const RhsState& s = st[q];
  const int mask = s.xmask & ((1 << len) - 1);
  const bool run = s.status == ST_RUN;
  if (!mask && !run) return;
  int m = 0;   // last iteration that took its step
  for (int i = 0; i < len; ++i)
    if (mask >> i & 1) m = i;
  T al[kGroupSlots];
#pragma unroll
  for (int i = 0; i < kGroupSlots; ++i) al[i] = (T)s.alpha_hist[i];
  const T be = (T)s.beta;
  SX* xr = x + (long)q * rs;
  const SR* rr = r + (long)q * rs;
  SP* pr = p0 + (long)q * rs;
  const SP* lastp = pr + (long)(run ? len - 1 : m) * ps;
  const bool copy = run || m > 0;
  constexpr int E = ChunkWidth<SX, SR, SP>::e;
  const long nt = vec ? n / TILE : 0;
  const int lane = threadIdx.x & 63;
  const long t1 = nt * (bx + 1) / NB;
  for (long t = nt * bx / NB + (threadIdx.x >> 6); t < t1; t += RT / 64) {
#pragma unroll
    for (int jj = 0; jj < 8 / E; ++jj) {
      const long i = t * TILE + jj * 64 * E + lane * E;
      T xv[E], pv[E];
      Chunk<SX, E>::ld(xr + i, xv);
      for (int g = 0; g < len; ++g) {
        if (!(mask >> g & 1)) continue;
        Chunk<SP, E>::ld(pr + (long)g * ps + i, pv);
#pragma unroll
        for (int k = 0; k < E; ++k) xv[k] = xv[k] + al[g] * pv[k];
      }
      Chunk<SX, E>::st(xr + i, xv);
      if (copy) {
        Chunk<SP, E>::ld(lastp + i, pv);
        if (run) {
          T rv[E];
          Chunk<SR, E>::ld(rr + i, rv);
#pragma unroll
          for (int k = 0; k < E; ++k) pv[k] = rv[k] + be * pv[k];
        }
        Chunk<SP, E>::st(pr + i, pv);
      }
    }
  }
  for (long i = TILE * nt + (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT) {
    T xv = (T)Store<SX>::to(xr[i]);
    for (int g = 0; g < len; ++g)
      if (mask >> g & 1) xv = xv + al[g] * (T)Store<SP>::to(pr[(long)g * ps + i]);
    xr[i] = Store<SX>::from(xv);
    if (copy) {
      const T pv = (T)Store<SP>::to(lastp[i]);
      pr[i] = Store<SP>::from(run ? (T)Store<SR>::to(rr[i]) + be * pv : pv);
    }
  }
}

// part[q*NB + bx] = sum of block bx's share of the n values v[q*n ...]
__device__ inline void k_sum_body(const double* __restrict__ v, long n, double* __restrict__ part,
    int bx, int NB, int q, double* sh) {
  const double* vr = v + (long)q * n;
  double acc = 0;
  for (long i = (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT) acc += vr[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)q * NB + bx] = t;
}

// ---- reliable update -------------------------------------------------------
// x_hi += x_lo / sigma ; x_lo = 0   (rhs that are running or waiting)
template <class SX>
__device__ inline void k_fold_x_body(double* __restrict__ xh, SX* __restrict__ xl,
                                               long n, long rs_h, long rs,
                                               const RhsState* __restrict__ st,
    int bx, int NB, int q, double* sh) {
  const RhsState& s = st[q];
  if (s.status != ST_UPDATE) return;
  const double inv = 1.0 / s.sigma;
  double* xr = xh + (long)q * rs_h;
  SX* lr = xl + (long)q * rs;
  for (long i = (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT) {
    xr[i] += (double)Store<SX>::to(lr[i]) * inv;
    lr[i] = Store<SX>::from(0);
  }
}

// r_hi = b - Ax ; partial |r_hi|^2 (also for finished rhs, for reporting)
__device__ inline void k_resid_body(const double* __restrict__ b,
                                              const double* __restrict__ Ax,
                                              double* __restrict__ rh, long n, long rs_b,
                                              long rs, double* __restrict__ part,
    int bx, int NB, int q, double* sh) {
  const double* br = b + (long)q * rs_b;
  const double* ar = Ax + (long)q * rs;
  double* rr = rh + (long)q * rs;
  double acc = 0;
  for (long i = (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT) {
    const double v = br[i] - ar[i];
    rr[i] = v;
    acc += v * v;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(long)q * NB + bx] = t;
}

// decide after the true residual: converged, or restart the inner recursion
__device__ inline void k_ru_decide_body(const double* __restrict__ part, int NB,
                                                  RhsState* __restrict__ st, double tol2,
                                                  double nreal, int scale, int first,
    int q, double* sh) {
  const double rr_true = part_sum(part, NB, q, sh);
  if (threadIdx.x) return;
  RhsState& s = st[q];
  // only right-hand sides that asked for an update take it, so a batched
  // solve follows exactly the trajectory each right-hand side has alone
  if (s.status != ST_UPDATE) return;
  s.rr_true = rr_true;
  s.first = 0;
  if (first) {
    // initial residual: p starts as r
    s.w_r = 1.0;
    s.beta = 0.0;
  } else {
    // the paused step still owes its p update: beta from the true residual
    s.ru += 1;
    const double rr_prev_phys = s.rr_prev / (s.sigma * s.sigma);
    s.w_r = 1.0;
    s.beta = rr_true / rr_prev_phys;
  }
  s.fresh = 1;
  if (!isfinite(rr_true)) {
    s.status = ST_NAN;
    return;
  }
  if (rr_true <= tol2 * s.bb) {
    s.status = ST_DONE;
    return;
  }
  if (s.final) {
    s.status = ST_NOTCONV;
    return;
  }
  const double sig = scale ? sqrt(nreal / rr_true) : 1.0;
  s.sigma_ratio = first ? 0.0 : sig / s.sigma;
  s.sigma = sig;
  s.rr = sig * sig * rr_true;
  s.rr_ru = s.rr;
  s.thresh = tol2 * s.bb * sig * sig;
  s.status = ST_RUN;
}

// r_lo = sigma r_hi ; p = w_r sigma r_hi + beta sigma_ratio p
template <class SR, class SP>
__device__ inline void k_ru_apply_body(const double* __restrict__ rh,
                                                 SR* __restrict__ rl, SP* __restrict__ p, long n,
                                                 long rs, const RhsState* __restrict__ st,
    int bx, int NB, int q, double* sh) {
  const RhsState& s = st[q];
  if (s.status != ST_RUN || !s.fresh) return;
  typedef typename Store<SR>::compute T;
  const double sg = s.sigma, wr = s.w_r, bs = s.beta * s.sigma_ratio;
  const double* hr = rh + (long)q * rs;
  SR* lr = rl + (long)q * rs;
  SP* pr = p + (long)q * rs;
  for (long i = (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT) {
    const double v = sg * hr[i];
    lr[i] = Store<SR>::from((T)v);
    const double pv = (bs != 0.0) ? bs * (double)Store<SP>::to(pr[i]) : 0.0;
    pr[i] = Store<SP>::from((typename Store<SP>::compute)(wr * v + pv));
  }
}

__device__ inline void k_init_state_body(RhsState* st, const double* part, int NB, int max_iter,
    int q, double* sh) {
  // bb from the partials of |b|^2
  const double bb = part_sum(part, NB, q, sh);
  if (threadIdx.x) return;
  RhsState& s = st[q];
  RhsState z = {};
  s = z;
  s.bb = bb;
  s.sigma = 1.0;
  s.first = 1;
  s.max_iter = max_iter;
  s.status = !isfinite(bb) ? ST_NAN : (bb > 0.0 ? ST_UPDATE : ST_DONE);
}

template <class S>
__device__ inline void k_zero_body(S* __restrict__ x, long n, long rs,
    int bx, int NB, int q, double* sh) {
  S* xr = x + (long)q * rs;
  for (long i = (long)bx * RT + threadIdx.x; i < n; i += (long)NB * RT)
    xr[i] = Store<S>::from(0);
}

}  // namespace qdwf
