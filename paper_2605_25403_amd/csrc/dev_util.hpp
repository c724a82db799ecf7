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

// Global-memory view of a generic pointer. Pointers read from the group
// structs are generic, and loads through them compile to flat instructions,
// which count against both the vector and the scalar wait counters, so every
// wait for a scalar load drains them too. Through this view they are global
// loads and stores, counted by the vector counter only: a kernel can issue
// all of its independent loads before its first wait.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> G(T* p) {
  return (gptr<T>)p;
}

// Sum over an aligned group of G lanes (G a power of two <= 64); every lane
// of the group receives the result.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<64>(v); }

// DPP lane move of a double (two 32-bit moves), CTRL a DPP control code.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over the 64 lanes of a wavefront, the same in every lane: a fixed
// pairwise tree with no round trip through LDS. Quads by two quad
// permutations ([1,0,3,2], then [2,3,0,1]), the four quads of each row of 16
// lanes by rotations of 4 and 8 lanes (lane 0 of a row then holds
// (Q0 + Q1) + (Q2 + Q3)), and the four rows from lanes 0, 16, 32, 48.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_d<0xb1>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4e>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);   // row_ror 4
  v += dpp_d<0x128>(v);   // row_ror 8
  return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

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

// Block sum over a compile-time block size BS (BS/64 waves); same contract as
// block_sum_n. sh needs (BS/64)*N doubles.
template <int BS, int N>
__device__ __forceinline__ void block_sum_t(double (&v)[N], double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int n = 0; n < N; ++n) v[n] = wave_total(v[n]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int n = 0; n < N; ++n) sh[wid * N + n] = v[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < BS / 64; ++q) s += sh[q * N + n];
    v[n] = s;
  }
}

// Partial sums are stored structure-of-arrays: value k of system j from
// producer block b is part[(j*KP + k)*nb + b], so a wavefront reading one
// value of 64 consecutive blocks makes one coalesced 512-byte load.
__device__ __forceinline__ size_t part_index(int j, int k, int nb, int b) {
  return ((size_t)(j * KP + k)) * nb + b;
}

// This thread's share of the partial sums of a producer kernel with nb
// blocks (nb <= KBS * KPART_Q): blocks tid, tid + KBS, ... summed in order.
// Records are loaded four per thread at a time from always-valid (clamped)
// addresses before any of them is used, so the loads of a chunk overlap each
// other and the caller's own independent loads; records past nb add zero.
// Value k of system j lands in v[j*K + k]; block_sum_t then gives the totals.
template <int NS, int K>
__device__ __forceinline__ void load_partials(const double* part, int nb, double* v) {
  constexpr int QC = 4;
#pragma unroll
  for (int n = 0; n < NS * K; ++n) v[n] = 0.0;
  const gptr<const double> P = G(part);
  for (int q0 = 0; q0 * KBS < nb; q0 += QC) {
    double x[QC][NS * K];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int b = (int)threadIdx.x + (q0 + q) * KBS;
      const int bc = b < nb ? b : nb - 1;
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) x[q][j * K + k] = P[part_index(j, k, nb, bc)];
    }
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const bool ok = (int)threadIdx.x + (q0 + q) * KBS < nb;
#pragma unroll
      for (int n = 0; n < NS * K; ++n) v[n] += ok ? x[q][n] : 0.0;
    }
  }
}

// load_partials in two steps, for kernels that issue other loads in between:
// partials_first loads this thread's first chunk (QC records) without using
// it, partials_rest adds that chunk and then the remaining ones, in the order
// of load_partials (same totals, bitwise).
template <int NS, int K>
__device__ __forceinline__ void partials_first(const double* part, int nb,
                                               double (&x)[4][NS * K]) {
  const gptr<const double> P = G(part);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = (int)threadIdx.x + q * KBS;
    const int bc = b < nb ? b : nb - 1;
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) x[q][j * K + k] = P[part_index(j, k, nb, bc)];
  }
}
template <int NS, int K>
__device__ __forceinline__ void partials_rest(const double* part, int nb,
                                              const double (&x)[4][NS * K], double* v) {
  constexpr int QC = 4;
#pragma unroll
  for (int n = 0; n < NS * K; ++n) v[n] = 0.0;
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const bool ok = (int)threadIdx.x + q * KBS < nb;
#pragma unroll
    for (int n = 0; n < NS * K; ++n) v[n] += ok ? x[q][n] : 0.0;
  }
  const gptr<const double> P = G(part);
  for (int q0 = QC; q0 * KBS < nb; q0 += QC) {
    double y[QC][NS * K];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int b = (int)threadIdx.x + (q0 + q) * KBS;
      const int bc = b < nb ? b : nb - 1;
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int k = 0; k < K; ++k) y[q][j * K + k] = P[part_index(j, k, nb, bc)];
    }
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const bool ok = (int)threadIdx.x + (q0 + q) * KBS < nb;
#pragma unroll
      for (int n = 0; n < NS * K; ++n) v[n] += ok ? y[q][n] : 0.0;
    }
  }
}

// Block-reduce acc[j*K + k] (KBS threads) and store them as the partials of
// block lb of a kernel with nb blocks.
template <int NS, int K>
__device__ __forceinline__ void store_partials(double* acc, double* part, int nb, int lb,
                                               double* sh) {
  double v[NS * K];
#pragma unroll
  for (int n = 0; n < NS * K; ++n) v[n] = acc[n];
  block_sum_t<KBS, NS * K>(v, sh);
  if (threadIdx.x < NS * K) {
    const int j = threadIdx.x / K, k = threadIdx.x % K;
    double val = 0.0;
#pragma unroll
    for (int q = 0; q < NS * K; ++q) val = (q == (int)threadIdx.x) ? v[q] : val;
    G(part)[part_index(j, k, nb, lb)] = val;
  }
}

__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

}  // namespace ipcs
