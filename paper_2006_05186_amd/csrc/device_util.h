// Small device helpers: complex arithmetic on (re, im) pairs, wave64 and
// workgroup reductions.
#pragma once
#include <type_traits>
#include "internal.h"

namespace cqm {

// Global-memory view of a generic pointer: loads through it compile to
// global (not flat) loads, which count only against vmcnt and so do not make
// waits for scalar or LDS traffic wait for them as well.  (The host pass of
// the same source sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define CQM_GLOBAL __attribute__((address_space(1)))
#else
#define CQM_GLOBAL
#endif
template <typename T> __device__ __forceinline__ const CQM_GLOBAL T* as_global(const T* p) {
  return (const CQM_GLOBAL T*)p;
}
template <typename T> __device__ __forceinline__ CQM_GLOBAL T* as_global(T* p) {
  return (CQM_GLOBAL T*)p;
}

template <typename R> __device__ __forceinline__ cplx<R> cmake(R re, R im) {
  cplx<R> z;
  z.re = re;
  z.im = im;
  return z;
}

// Partner value for the exchange between lanes l and l ^ OFF: DPP moves
// within a row of 16 lanes for OFF = 1, 2, 8 (VALU, no LDS traffic), an LDS
// swizzle for 4 and 16, a permute for 32.
template <int OFF> __device__ __forceinline__ int xor_lane_i(int v) {
  if constexpr (OFF == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad [1,0,3,2]
  else if constexpr (OFF == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad [2,3,0,1]
  else if constexpr (OFF == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row rotate 8
  else if constexpr (OFF == 4 || OFF == 16) return __builtin_amdgcn_ds_swizzle(v, 0x1F | (OFF << 10));
  else return __shfl_xor(v, OFF, 64);
}
template <int OFF> __device__ __forceinline__ double xor_lane(double v) {
  const int lo = xor_lane_i<OFF>(__double2loint(v));
  const int hi = xor_lane_i<OFF>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int OFF> __device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane_i<OFF>(__float_as_int(v)));
}

// Sum of NV (<= 64) per-lane values over the 64 lanes of a wave, scattered:
// on return lane l holds, in a[0], the total of entry scatter_entry<NV>(l)
// (lanes that differ only in bits >= log2 NV hold the same entry).  The
// exchanges go from the nearest lanes outwards, so the levels that move the
// most values are DPP moves.
template <int NV, int OFF = 1, typename T>
__device__ __forceinline__ void wave_reduce_scatter_near(T* a, int lane) {
  if constexpr (NV > 1) {
    constexpr int H = NV / 2;
    const bool up = (lane & OFF) != 0;
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const T send = up ? a[u] : a[u + H];
      const T keep = up ? a[u + H] : a[u];
      a[u] = keep + xor_lane<OFF>(send);
    }
    wave_reduce_scatter_near<H, OFF * 2, T>(a, lane);
  } else if constexpr (OFF < 64) {
    a[0] += xor_lane<OFF>(a[0]);
    wave_reduce_scatter_near<1, OFF * 2, T>(a, lane);
  }
}
// Double-double value hi + lo (|lo| <= ulp(hi)/2): sums of FP64 products
// carried to about 106 bits (error-free product by fma, Knuth's two-sum).
struct dd {
  double hi, lo;
};
__device__ __forceinline__ dd two_prod(double a, double b) {
  const double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__device__ __forceinline__ dd operator+(dd a, dd b) {
  const double s = a.hi + b.hi;
  const double bb = s - a.hi;
  double e = (a.hi - (s - bb)) + (b.hi - bb);  // two-sum error of a.hi + b.hi
  e += a.lo + b.lo;
  const double h = s + e;
  return dd{h, e - (h - s)};
}
__device__ __forceinline__ dd operator-(dd a) { return dd{-a.hi, -a.lo}; }
__device__ __forceinline__ dd& operator+=(dd& a, dd b) {
  a = a + b;
  return a;
}
template <int OFF> __device__ __forceinline__ dd xor_lane(dd v) {
  return dd{xor_lane<OFF>(v.hi), xor_lane<OFF>(v.lo)};
}

template <typename T> __device__ __forceinline__ T wave_sum_near(T v) {
  T a[1] = {v};
  wave_reduce_scatter_near<1, 1, T>(a, 0);
  return a[0];
}
// value of lane `src` (wave-uniform) in every lane
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
// entry whose total lane l holds after wave_reduce_scatter_near<NV>: bit b of
// the lane (from b = 0) selected the upper half at the level with NV >> b
// values
template <int NV> __device__ __forceinline__ int scatter_entry(int lane) {
  int e = 0;
#pragma unroll
  for (int b = 0, h = NV / 2; h >= 1; ++b, h >>= 1)
    if (lane & (1 << b)) e += h;
  return e;
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  if constexpr (std::is_same_v<T, float> || std::is_same_v<T, double>) {
    return wave_sum_near(v);
  } else {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  }
}


// Row i of a stored-operator product from its tile partial sums:
// y_i = sum_{Y < nt} P[Y][i] in a fixed order (P: nt slots of nt kSymB rows).
template <typename R>
__device__ __forceinline__ cplx<R> sym_row_sum(const cplx<R>* __restrict__ P, int M, int i) {
  const int nt = sym_blocks(M), ntB = nt * kSymB;
  R re = R(0), im = R(0);
  for (int Y0 = 0; Y0 < nt; Y0 += 8) {
    // eight loads in flight (clamped indices), added in slot order
    cplx<R> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)min(Y0 + u, nt - 1) * ntB + i];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (Y0 + u < nt) {
        re += v[u].re;
        im += v[u].im;
      }
  }
  cplx<R> o;
  o.re = re;
  o.im = im;
  return o;
}

// sum_{q < S} P[q * stride] (doubles) in slot order, eight loads in flight.
__device__ __forceinline__ double slot_sum(const double* __restrict__ P, int S, int64_t stride) {
  double acc = 0.0;
  for (int q0 = 0; q0 < S; q0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)min(q0 + u, S - 1) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q0 + u < S) acc += v[u];
  }
  return acc;
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

// Block-Jacobi application to one kSymB-row block by one wave: lane r adds
// sum_c P[c][r] v_c.  The stored inverse of a complex symmetric block is
// symmetric up to rounding; every application (inner steps and the update
// of x) uses this one orientation, so the preconditioner is one fixed
// matrix.  p holds the block's entries P[c][lane] (column-major for lane r),
// vb the block of v in LDS; A is the accumulation type.
template <typename R, typename A>
__device__ __forceinline__ void pblock_acc(const cplx<R> (&p)[kSymB], const cplx<A>* vb, A& re,
                                           A& im) {
#pragma unroll
  for (int c = 0; c < kSymB; ++c) {
    const cplx<A> v = vb[c];
    re += (A)p[c].re * v.re - (A)p[c].im * v.im;
    im += (A)p[c].re * v.im + (A)p[c].im * v.re;
  }
}
template <typename R>
__device__ __forceinline__ void pblock_load(const cplx<R>* __restrict__ Pb, int lane,
                                            cplx<R> (&p)[kSymB]) {
#pragma unroll
  for (int c = 0; c < kSymB; ++c) p[c] = as_global(Pb)[c * kSymB + lane];
}
// The same sum with the entries loaded NC columns at a time (FP64 blocks:
// register budget).
template <typename R, typename A, int NC>
__device__ __forceinline__ void pblock_mul(const cplx<R>* __restrict__ Pb, const cplx<A>* vb,
                                           int lane, A& re, A& im) {
  for (int c0 = 0; c0 < kSymB; c0 += NC) {
    cplx<R> p[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) p[u] = as_global(Pb)[(c0 + u) * kSymB + lane];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const cplx<A> v = vb[c0 + u];
      re += (A)p[u].re * v.re - (A)p[u].im * v.im;
      im += (A)p[u].re * v.im + (A)p[u].im * v.re;
    }
  }
}

}  // namespace cqm
