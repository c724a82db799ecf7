// Device helpers: lane-group and block reductions, and the fence-free
// two-stage reduction used for dot products.
//
// Cross-block reductions never synchronize blocks inside a kernel: a producer
// kernel writes one partial sum per block, and every block of the next kernel
// (after the kernel boundary has made the partials visible) sums all of them in
// block order with a fixed tree. The result is deterministic, identical in
// every consumer block, and independent of which other systems share a launch.
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

// Sum over the block (blockDim.x a multiple of 64, at most 1024); result valid
// in every thread; fixed order of additions. sh needs blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += sh[w];
  return s;
}

// Sums N values over the block at once (one barrier pair): out[n] valid in
// every thread, fixed order of additions. sh needs 16*N doubles.
template <int N>
__device__ __forceinline__ void block_sum_n(const double (&v)[N], double (&out)[N], double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double w[N];
#pragma unroll
  for (int n = 0; n < N; ++n) w[n] = wave_sum(v[n]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int n = 0; n < N; ++n) sh[wid * N + n] = w[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
    for (int q = 0; q < nw; ++q) s += sh[q * N + n];
    out[n] = s;
  }
}

// Partial sums of a producer kernel, loaded in two phases so the loads can
// be issued early and overlap other memory traffic: load() only fetches this
// thread's entries (producer blocks tid, tid + blockDim, ...), reduce() sums
// them over the block in a fixed order. tot[j][k] = sum over b < nb of
// part[(b*GMAX + j)*KP + k] for j < ns, k < K; valid in every thread.
template <int K>
struct Partials {
  double v[GMAX][K];
  __device__ __forceinline__ void load(const double* part, int nb, int ns) {
#pragma unroll
    for (int j = 0; j < GMAX; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) v[j][k] = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      const double* p = part + (size_t)b * GMAX * KP;
#pragma unroll
      for (int j = 0; j < GMAX; ++j)
        if (j < ns)
#pragma unroll
          for (int k = 0; k < K; ++k) v[j][k] += p[j * KP + k];
    }
  }
  __device__ __forceinline__ void reduce(int ns, double (&tot)[GMAX][K], double* sh) const {
    double flat[GMAX * K], out[GMAX * K];
#pragma unroll
    for (int j = 0; j < GMAX; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) flat[j * K + k] = j < ns ? v[j][k] : 0.0;
    block_sum_n<GMAX * K>(flat, out, sh);
#pragma unroll
    for (int j = 0; j < GMAX; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) tot[j][k] = out[j * K + k];
  }
};

// Block-reduce acc[j][k] and store them as this block's partials.
template <int K>
__device__ __forceinline__ void store_partials(const double (&acc)[GMAX][K], int ns, double* part,
                                               int lb, double* sh) {
  double flat[GMAX * K], out[GMAX * K];
#pragma unroll
  for (int j = 0; j < GMAX; ++j)
#pragma unroll
    for (int k = 0; k < K; ++k) flat[j * K + k] = acc[j][k];
  block_sum_n<GMAX * K>(flat, out, sh);
  if (threadIdx.x < GMAX * K) {
    const int j = threadIdx.x / K, k = threadIdx.x % K;
    double val = 0.0;
#pragma unroll
    for (int q = 0; q < GMAX * K; ++q) val = (q == (int)threadIdx.x) ? out[q] : val;
    if (j < ns) part[((size_t)lb * GMAX + j) * KP + k] = val;
  }
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

}  // namespace ipcs
