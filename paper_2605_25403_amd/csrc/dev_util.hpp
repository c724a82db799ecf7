// Device helpers: lane-group and block reductions, and the deterministic
// "last block finishes the reduction" pattern used for dot products.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace ipcs {

// Sum over an aligned group of G lanes (G a power of two <= 64); every lane
// of the group receives the result.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// Sum over the block (blockDim.x == BLOCK); result valid in every thread.
// The order of additions is fixed, so the result is deterministic.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) s += sh[w];
  return s;
}

// Each block contributes K partial sums; the last block to arrive reduces all
// blocks' partials in block order and returns true (in all its threads) with
// the totals in tot[]. Other blocks return false. The reduction order depends
// only on nblk, never on arrival order, so results are bitwise reproducible.
template <int K>
__device__ __forceinline__ bool reduce_last(const double (&v)[K], double* part, uint32_t* cnt,
                                            int nblk, int lb, double (&tot)[K]) {
  __shared__ double sh[BLOCK / 64];
  __shared__ int last;
  double bs[K];
#pragma unroll
  for (int k = 0; k < K; ++k) bs[k] = block_sum(v[k], sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) part[(size_t)lb * KPART + k] = bs[k];
    __threadfence();
    uint32_t prev = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == uint32_t(nblk - 1));
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nblk; i += BLOCK)
      a += __hip_atomic_load(&part[(size_t)i * KPART + k], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    tot[k] = block_sum(a, sh);
  }
  if (threadIdx.x == 0) *cnt = 0u;
  return true;
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

}  // namespace ipcs
