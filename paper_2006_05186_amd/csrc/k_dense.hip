// Stored dense operator: y_l = V_l x_l for every active frequency system,
// V_l an M x M row-major complex matrix in HBM.  Bandwidth bound: one wave per
// row, four independent loads in flight per lane, x_l served from cache.
#include "device_util.h"

namespace cqm {

template <typename R>
__global__ __launch_bounds__(256) void k_dense_gemv(const cplx<R>* __restrict__ V, int M,
                                                    const cplx<R>* __restrict__ x, int64_t xs,
                                                    cplx<R>* __restrict__ y, int64_t ys,
                                                    const int* __restrict__ active) {
  const int l = blockIdx.y;
  if (active && !active[l * kSysiStride]) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;
  const cplx<R>* row = V + ((int64_t)l * M + i) * M;
  const cplx<R>* xv = x + (int64_t)l * xs;
  R re = R(0), im = R(0);
  int j = lane;
  for (; j + 192 < M; j += 256) {
    cplx<R> a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = row[j + 64 * u];
      b[u] = xv[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      re += a[u].re * b[u].re - a[u].im * b[u].im;
      im += a[u].re * b[u].im + a[u].im * b[u].re;
    }
  }
  for (; j < M; j += 64) {
    const cplx<R> a = row[j], b = xv[j];
    re += a.re * b.re - a.im * b.im;
    im += a.re * b.im + a.im * b.re;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    cplx<R> o;
    o.re = re;
    o.im = im;
    y[(int64_t)l * ys + i] = o;
  }
}

template <typename R>
void launch_dense_gemv(const cplx<R>* V, int M, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y,
                       int64_t ys, const int* active, hipStream_t s) {
  dim3 grid((M + 3) / 4, nsys);
  hipLaunchKernelGGL((k_dense_gemv<R>), grid, dim3(256), 0, s, V, M, x, xs, y, ys, active);
  CQM_HIP(hipGetLastError());
}

// Products over system descriptors (systems of several problems, different
// sizes): one workgroup per (system, 4 rows).
template <typename R>
__global__ __launch_bounds__(256) void k_dense_gemv_desc(const SysDesc* __restrict__ sd,
                                                         const RowBlock* __restrict__ map, int which,
                                                         int j) {
  const RowBlock rb = map[blockIdx.x];
  const SysDesc D = sd[rb.sys];
  if (which == 0 ? !D.sysi[1] : !D.sysi[0]) return;
  const int lane = threadIdx.x & 63;
  const int i = rb.row0 + (threadIdx.x >> 6);
  const int M = D.M;
  if (i >= M) return;
  const cplx<R>* V;
  const cplx<R>* xv;
  cplx<R>* y;
  if (which == 0) {
    V = (const cplx<R>*)(sizeof(R) == 4 ? D.V32 : (const void*)D.V64);
    xv = (const cplx<R>*)D.basis + (int64_t)j * M;
    y = (cplx<R>*)D.basis + (int64_t)(j + 1) * M;
  } else {
    V = (const cplx<R>*)(const void*)D.V64;
    xv = (const cplx<R>*)(const void*)D.x;
    y = (cplx<R>*)(void*)D.r;
  }
  const cplx<R>* row = V + (int64_t)i * M;
  R re = R(0), im = R(0);
  int jj = lane;
  for (; jj + 192 < M; jj += 256) {
    cplx<R> a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = row[jj + 64 * u];
      b[u] = xv[jj + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      re += a[u].re * b[u].re - a[u].im * b[u].im;
      im += a[u].re * b[u].im + a[u].im * b[u].re;
    }
  }
  for (; jj < M; jj += 64) {
    const cplx<R> a = row[jj], b = xv[jj];
    re += a.re * b.re - a.im * b.im;
    im += a.re * b.im + a.im * b.re;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    cplx<R> o;
    o.re = re;
    o.im = im;
    y[i] = o;
  }
}

template <typename R>
void launch_dense_gemv_desc(const SysDesc* sd, const RowBlock* map, int nblocks, int which, int j,
                            hipStream_t s) {
  hipLaunchKernelGGL((k_dense_gemv_desc<R>), dim3(nblocks), dim3(256), 0, s, sd, map, which, j);
  CQM_HIP(hipGetLastError());
}
template void launch_dense_gemv_desc<float>(const SysDesc*, const RowBlock*, int, int, int, hipStream_t);
template void launch_dense_gemv_desc<double>(const SysDesc*, const RowBlock*, int, int, int, hipStream_t);

template void launch_dense_gemv<float>(const cf32*, int, int, const cf32*, int64_t, cf32*, int64_t,
                                       const int*, hipStream_t);
template void launch_dense_gemv<double>(const cf64*, int, int, const cf64*, int64_t, cf64*,
                                        int64_t, const int*, hipStream_t);

}  // namespace cqm
