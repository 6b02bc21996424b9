// The Domain Wall kernel launched over one context: the 4D Wilson hop D_h on
// every slice of the fifth dimension fused with the Mobius 5D factors and the
// 4D-local epilogue (the body and its work decomposition are in hopbody.h).
#include <cstdlib>
#include <type_traits>

#include "hopbody.h"

namespace qdwf {

namespace {

// Waves per SIMD of a launch: the one-parity hops (D_eo and the solver's
// M_pc stages) in FP32 with the interleaved layout run at three (132-138
// registers, no spills), which measured 2-4 % faster than two; the full
// operator over both parities keeps two, at three it measured 5 % slower.
template <class S, int LAYOUT, bool DPP16, bool ONEPAR> struct HopWaves {
  static constexpr int v = (std::is_same<S, float>::value && LAYOUT == QDWF_RIRI && ONEPAR)
                               ? 3 : WavesPerEU<S, LAYOUT, DPP16>::v;
};

template <class S, int LAYOUT, bool DAG, bool DPP16, bool MINV, bool CHI, bool ONEPAR>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(HopWaves<S, LAYOUT, DPP16, ONEPAR>::v,
                                   HopWaves<S, LAYOUT, DPP16, ONEPAR>::v)))
hop_kernel(HopK k) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the XCD remap hands each XCD a contiguous range of logical blocks
  const int L = k.xcd ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  hop_block<S, LAYOUT, DAG, DPP16, MINV, CHI>(k, L, smem);
}

template <class S, int LAYOUT, bool DAG, bool DPP16, bool MINV, bool CHI>
int run_hop_k(qdwf_ctx* ctx, int prec, const HopArgs& a, hipStream_t st, const HopShape& sh) {
  HopK k;
  size_t lds = 0;
  int nb = 0;
  int rc = make_hopk<S, MINV>(ctx, prec, a, sh, &k, &lds, &nb);
  if (rc) return rc;
  // only FP32 in the interleaved layout has a one-parity form of its own;
  // M_ee^-1 and chi hops are one-parity by construction
  if constexpr (std::is_same<S, float>::value && LAYOUT == QDWF_RIRI) {
    if (MINV || CHI || a.npar == 1)
      hipLaunchKernelGGL((hop_kernel<S, LAYOUT, DAG, DPP16, MINV, CHI, true>), dim3(nb),
                         dim3(sh.threads), lds, st, k);
    else if constexpr (!MINV && !CHI)
      hipLaunchKernelGGL((hop_kernel<S, LAYOUT, DAG, DPP16, MINV, CHI, false>), dim3(nb),
                         dim3(sh.threads), lds, st, k);
  } else {
    hipLaunchKernelGGL((hop_kernel<S, LAYOUT, DAG, DPP16, MINV, CHI, false>), dim3(nb),
                       dim3(sh.threads), lds, st, k);
  }
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

template <class S, int LAYOUT, bool DAG>
int run_hop(qdwf_ctx* ctx, int prec, const HopArgs& a, hipStream_t st, const HopShape& sh) {
  if (a.chi && DAG) return fail(QDWF_EINVAL, "the adjoint hop takes no A-applied input");
  if constexpr (!DAG) {
    if (a.chi) {
      if (ctx->g.Ls == 16)
        return a.minv ? run_hop_k<S, LAYOUT, false, true, true, true>(ctx, prec, a, st, sh)
                      : run_hop_k<S, LAYOUT, false, true, false, true>(ctx, prec, a, st, sh);
      if (a.minv) return fail(QDWF_EINVAL, "fused M_ee^-1 needs Ls = 16");
      return run_hop_k<S, LAYOUT, false, false, false, true>(ctx, prec, a, st, sh);
    }
  }
  if (ctx->g.Ls == 16)
    return a.minv ? run_hop_k<S, LAYOUT, DAG, true, true, false>(ctx, prec, a, st, sh)
                  : run_hop_k<S, LAYOUT, DAG, true, false, false>(ctx, prec, a, st, sh);
  if (a.minv) return fail(QDWF_EINVAL, "fused M_ee^-1 needs Ls = 16");
  return run_hop_k<S, LAYOUT, DAG, false, false, false>(ctx, prec, a, st, sh);
}

}  // namespace

HopShape default_shape(const qdwf_ctx* ctx, int prec, int nrhs) {
  HopShape sh;
  // at most 32 (site, rhs) groups per block: bounds the LDS link stage
  // (32 sites x 8 links x 18 reals, 36 KB in FP64) for every Ls
  const int gpw = 64 / ctx->g.Ls;
  int waves = 32 / gpw;
  if (waves < 1) waves = 1;
  if (waves > 4) waves = 4;
  sh.threads = 64 * waves;
  sh.xcd = 1;
  // one right-hand side per block: with the right-hand sides outermost in the
  // block order this measured faster than sharing the staged links between
  // several right-hand sides of a block (the tuner still tries both)
  sh.nrb = 1;
  sh.lds_pad = 0;
  // the t-sweep of the full operator: measured faster than the checkerboard
  // traversal in FP32 with 16- and 32-wide rows (one and two blocks of 8
  // waves per CU); slower with 24-wide ones (6 waves per CU), in BF16
  // storage, and in FP16 storage since the checkerboard kernel keeps FP16
  // neighbours packed (32^4 x 16 D 0.73 against 0.84 ms); the tuner tries
  // it wherever it applies
  const int Lx = ctx->g.L[0];
  sh.sweep = (prec == QDWF_F32 && (Lx == 16 || Lx == 32)) ? 1 : 0;
  if (const char* e = std::getenv("QDWF_HOP_LDS_PAD")) sh.lds_pad = std::atoi(e);
  if (const char* e = std::getenv("QDWF_HOP_THREADS")) {
    const int t = std::atoi(e);
    if (t >= 64 && t <= 256 && t % 64 == 0) sh.threads = t;
  }
  (void)nrhs;
  return sh;
}

int launch_hop(qdwf_ctx* ctx, int prec, int layout, int dagger, const HopArgs& a,
               hipStream_t st, const HopShape* shape) {
  HopShape sh;
  if (shape) sh = *shape;
  else if (!tuned_shape(ctx, prec, layout, dagger, a.nrhs, &sh)) sh = default_shape(ctx, prec, a.nrhs);
  const int G = (sh.threads / 64) * (64 / ctx->g.Ls);
  if (sh.threads % 64 || sh.threads < 64 || sh.threads > 256 || sh.nrb < 1 || G % sh.nrb)
    return fail(QDWF_EINVAL, "invalid hop launch shape (threads %d, nrb %d)", sh.threads, sh.nrb);
  // the full operator on one whole field takes the t-sweep where it applies
  // (QDWF_SWEEP=1 / 0 forces it on / off where it applies)
  const char* force = std::getenv("QDWF_SWEEP");
  const bool sweep = (force && *force) ? force[0] == '1' : sh.sweep != 0;
  if (sweep && sweep_eligible(ctx, prec, layout, a)) return launch_sweep(ctx, prec, dagger, a, st);
  auto go = [&](auto tag_s) -> int {
    typedef decltype(tag_s) S;
    if (layout == QDWF_RIRI) {
      return dagger ? run_hop<S, QDWF_RIRI, true>(ctx, prec, a, st, sh)
                    : run_hop<S, QDWF_RIRI, false>(ctx, prec, a, st, sh);
    }
    return dagger ? run_hop<S, QDWF_RRII, true>(ctx, prec, a, st, sh)
                  : run_hop<S, QDWF_RRII, false>(ctx, prec, a, st, sh);
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
