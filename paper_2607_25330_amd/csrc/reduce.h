// Block partial sums for the BiCGSTAB inner products.
//
// A kernel that contributes to an inner product accumulates FP64 sums per
// thread, reduces them over its block (wave shuffles, then LDS) and writes
// one partial per block to part[block * KPART + k].  A one-block finalize
// kernel adds the partials in a fixed order, so results are deterministic
// and need no grid-wide fence: the launch boundary orders the two kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace psfd {

constexpr int KPART = 4;  // stride of one block's partials

template <int NV, int NT>
__device__ __forceinline__ void block_partials(double (&acc)[NV], double* __restrict__ part) {
  static_assert(NT % 64 == 0, "block size must be a multiple of the wavefront");
  __shared__ double sm[NV][NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sm[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) s += sm[k][w];
      part[(size_t)blockIdx.x * KPART + k] = s;
    }
  }
}

}  // namespace psfd
