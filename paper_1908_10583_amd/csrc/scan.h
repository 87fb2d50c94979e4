// Block-wide scans and reductions for 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>

namespace fora {

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Exclusive scan over the block (blockDim.x a multiple of 64, at most 1024).
// s_tmp needs blockDim.x / 64 entries. Returns the exclusive prefix; `total`
// receives the block sum. Contains two __syncthreads().
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* s_tmp, T& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const T inc = wave_inclusive_scan(v);
  if (lane == 63) s_tmp[wid] = inc;
  __syncthreads();
  T base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    const T t = s_tmp[w];
    if (w < wid) base += t;
    tot += t;
  }
  total = tot;
  __syncthreads();
  return base + inc - v;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* s_tmp) {
  T total;
  (void)block_exclusive_scan(v, s_tmp, total);
  return total;
}

__device__ __forceinline__ unsigned lane_rank(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

}  // namespace fora
