// Streaming kernels for the memory-system probes: the per-site SU(3) matrix
// product of the Benchmark_su3 study in Section 4.2 (C(x) = A(x) B(x) for 3x3
// complex matrices, 198 real flops each) and the triad a = b + s c of the
// STREAM measurements in Section 3.
//
// A matrix is 18 reals (72 bytes in FP32, 144 in FP64), an awkward stride
// for per-lane vector loads, so the SU(3) kernel moves each block's tile of
// matrices between HBM and LDS with contiguous 16-byte loads and stores that
// span the whole tile, and every lane then reads its own matrices from LDS.
#include <algorithm>

#include "common.h"
#include "spin.h"

namespace qdwf {

namespace {

// Matrices per block (one per lane): the two LDS tiles take 36 KB either way.
template <class T> struct Su3Tile { static constexpr int n = sizeof(T) == 8 ? 128 : 256; };

// Copies `n` reals between global memory and LDS with 16-byte words where the
// tile is 16-byte aligned and whole (the common case), reals otherwise.
template <class T, bool TO_LDS>
__device__ inline void tile_copy(T* __restrict__ lds, T* __restrict__ g, long n, bool vec) {
  constexpr int W = 16 / sizeof(T);
  if (vec) {
    const long nv = n / W;
    for (long v = threadIdx.x; v < nv; v += blockDim.x) {
      if (TO_LDS) reinterpret_cast<uint4*>(lds)[v] = reinterpret_cast<const uint4*>(g)[v];
      else reinterpret_cast<uint4*>(g)[v] = reinterpret_cast<const uint4*>(lds)[v];
    }
    for (long r = nv * W + threadIdx.x; r < n; r += blockDim.x) {
      if (TO_LDS) lds[r] = g[r];
      else g[r] = lds[r];
    }
  } else {
    for (long r = threadIdx.x; r < n; r += blockDim.x) {
      if (TO_LDS) lds[r] = g[r];
      else g[r] = lds[r];
    }
  }
}

template <class T>
__global__ void __launch_bounds__(256) su3_mul_kernel(T* __restrict__ C, const T* __restrict__ A,
                                                      const T* __restrict__ B, long n) {
  constexpr int NT = Su3Tile<T>::n;
  __shared__ __align__(16) T sa[NT * 18];
  __shared__ __align__(16) T sb[NT * 18];
  const long m0 = (long)blockIdx.x * NT;
  const long cnt = min((long)NT, n - m0);
  const long nr = cnt * 18;
  // the tile starts at real m0 * 18; 16-byte aligned when m0 * 18 * sizeof(T) is
  const bool vec = ((m0 * 18 * (long)sizeof(T)) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(B) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(C) & 15) == 0;
  tile_copy<T, true>(sa, const_cast<T*>(A) + m0 * 18, nr, vec);
  tile_copy<T, true>(sb, const_cast<T*>(B) + m0 * 18, nr, vec);
  __syncthreads();
  if (threadIdx.x < cnt) {
    const T* a = sa + threadIdx.x * 18;
    const T* b = sb + threadIdx.x * 18;
    T a_[18], b_[18], c_[18];
#pragma unroll
    for (int r = 0; r < 18; ++r) { a_[r] = a[r]; b_[r] = b[r]; }
    // C[i][k] = sum_j A[i][j] B[j][k]: one multiply and five FMAs per real
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T* ai = a_ + 6 * i;
        T re = ai[0] * b_[2 * k], im = ai[0] * b_[2 * k + 1];
        re = fmac(-ai[1], b_[2 * k + 1], re);
        im = fmac(ai[1], b_[2 * k], im);
#pragma unroll
        for (int j = 1; j < 3; ++j) {
          const T* bj = b_ + 6 * j + 2 * k;
          re = fmac(ai[2 * j], bj[0], re);
          im = fmac(ai[2 * j], bj[1], im);
          re = fmac(-ai[2 * j + 1], bj[1], re);
          im = fmac(ai[2 * j + 1], bj[0], im);
        }
        c_[6 * i + 2 * k] = re;
        c_[6 * i + 2 * k + 1] = im;
      }
    T* c = sa + threadIdx.x * 18;   // the lane's own slot of the A tile
#pragma unroll
    for (int r = 0; r < 18; ++r) c[r] = c_[r];
  }
  __syncthreads();
  tile_copy<T, false>(sa, C + m0 * 18, nr, vec);
}

template <class T>
__global__ void __launch_bounds__(256) triad_kernel(T* __restrict__ a, const T* __restrict__ b,
                                                    const T* __restrict__ c, T s, long n, bool vec) {
  constexpr int W = 16 / sizeof(T);
  const long nv = vec ? n / W : 0;
  const long stride = (long)gridDim.x * blockDim.x;
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride) {
    T x[W], y[W], z[W];
    *reinterpret_cast<uint4*>(x) = reinterpret_cast<const uint4*>(b)[v];
    *reinterpret_cast<uint4*>(y) = reinterpret_cast<const uint4*>(c)[v];
#pragma unroll
    for (int w = 0; w < W; ++w) z[w] = fmac(s, y[w], x[w]);
    reinterpret_cast<uint4*>(a)[v] = *reinterpret_cast<const uint4*>(z);
  }
  for (long r = nv * W + (long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride)
    a[r] = fmac(s, c[r], b[r]);
}

}  // namespace

int launch_su3_mul(void* C, const void* A, const void* B, long n, int prec, hipStream_t st) {
  if (n == 0) return QDWF_OK;
  const int nt = prec == QDWF_F64 ? Su3Tile<double>::n : Su3Tile<float>::n;
  const long blocks = (n + nt - 1) / nt;
  if (blocks > 0x7fffffffL) return fail(QDWF_EINVAL, "too many matrices for one launch");
  if (prec == QDWF_F64)
    hipLaunchKernelGGL(su3_mul_kernel<double>, dim3((unsigned)blocks), dim3(nt), 0, st,
                       (double*)C, (const double*)A, (const double*)B, n);
  else
    hipLaunchKernelGGL(su3_mul_kernel<float>, dim3((unsigned)blocks), dim3(nt), 0, st,
                       (float*)C, (const float*)A, (const float*)B, n);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

int launch_triad(void* a, const void* b, const void* c, double s, long n, int prec,
                 hipStream_t st) {
  if (n == 0) return QDWF_OK;
  const bool vec = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) |
                    reinterpret_cast<uintptr_t>(c)) & 15) == 0;
  const long blocks = std::min<long>((n / 4 + 255) / 256 + 1, 256L * 1024);
  if (prec == QDWF_F64)
    hipLaunchKernelGGL(triad_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st, (double*)a,
                       (const double*)b, (const double*)c, s, n, vec);
  else
    hipLaunchKernelGGL(triad_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st, (float*)a,
                       (const float*)b, (const float*)c, (float)s, n, vec);
  QDWF_HIP(hipGetLastError());
  return QDWF_OK;
}

}  // namespace qdwf
