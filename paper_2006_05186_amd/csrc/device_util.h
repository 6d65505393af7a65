// Small device helpers: complex arithmetic on (re, im) pairs, wave64 and
// workgroup reductions.
#pragma once
#include "internal.h"

namespace cqm {

template <typename R> __device__ __forceinline__ cplx<R> cmake(R re, R im) {
  cplx<R> z;
  z.re = re;
  z.im = im;
  return z;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a workgroup of blockDim.x threads (multiple of 64, <= 1024).
// `red` is caller-provided shared scratch of >= 16 T; result broadcast to all.
template <typename T> __device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T t = T(0);
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

}  // namespace cqm
