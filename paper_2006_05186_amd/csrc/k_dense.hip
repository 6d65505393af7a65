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
// sizes): one workgroup per (group, 4 rows), one wave per row.  A group is a
// set of systems sharing the operator slice, so the row is read once and
// multiplied by every member's vector.
template <typename R>
__global__ __launch_bounds__(256) void k_dense_gemv_desc(const SysDesc* __restrict__ sd,
                                                         const GemvGroup* __restrict__ groups,
                                                         const RowBlock* __restrict__ map, int which,
                                                         int j, unsigned long long* ctr) {
  const RowBlock rb = map[blockIdx.x];
  const GemvGroup G = groups[rb.group];
  const SysDesc D0 = sd[G.sys[0]];
  const int M = D0.M;
  const int lane = threadIdx.x & 63;
  const int i = rb.row0 + (threadIdx.x >> 6);
  if (i >= M) return;
  const cplx<R>* xs[kMaxGroup];
  cplx<R>* ys[kMaxGroup];
  int n = 0;
  for (int q = 0; q < G.n; ++q) {
    const SysDesc& D = sd[G.sys[q]];
    if (which == 0 ? !D.sysi[1] : !D.sysi[0]) continue;
    if (which == 0) {
      xs[n] = (const cplx<R>*)D.basis + (int64_t)j * M;
      ys[n] = (cplx<R>*)D.basis + (int64_t)(j + 1) * M;
    } else {
      xs[n] = (const cplx<R>*)(const void*)D.x;
      ys[n] = (cplx<R>*)(void*)D.r;
    }
    ++n;
  }
  if (n == 0) return;
  if (ctr && threadIdx.x == 0 && rb.row0 == 0) {
    // algorithmic bytes of the whole product, charged once per group by its
    // first row block: the operator slice once, each member's input and
    // result vectors once
    const unsigned long long MM = (unsigned long long)M;
    atomicAdd(ctr, (MM * MM + (unsigned long long)n * 2 * MM) * sizeof(cplx<R>));
  }
  const cplx<R>* V = (which == 0) ? (const cplx<R>*)(sizeof(R) == 4 ? D0.V32 : (const void*)D0.V64)
                                  : (const cplx<R>*)(const void*)D0.V64;
  const cplx<R>* row = V + (int64_t)i * M;
  if (n == 1) {  // (single-member groups normally take k_dense_gemv_desc1)
    const cplx<R>* xv = xs[0];
    R sre = R(0), sim = R(0);
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
        sre += a[u].re * b[u].re - a[u].im * b[u].im;
        sim += a[u].re * b[u].im + a[u].im * b[u].re;
      }
    }
    for (; jj < M; jj += 64) {
      const cplx<R> a = row[jj], b = xv[jj];
      sre += a.re * b.re - a.im * b.im;
      sim += a.re * b.im + a.im * b.re;
    }
    sre = wave_sum(sre);
    sim = wave_sum(sim);
    if (lane == 0) {
      cplx<R> o;
      o.re = sre;
      o.im = sim;
      ys[0][i] = o;
    }
    return;
  }
  R re[kMaxGroup], im[kMaxGroup];
#pragma unroll
  for (int q = 0; q < kMaxGroup; ++q) re[q] = im[q] = R(0);
  for (int jj = lane; jj < M; jj += 64) {
    const cplx<R> a = row[jj];
#pragma unroll
    for (int q = 0; q < kMaxGroup; ++q)
      if (q < n) {
        const cplx<R> b = xs[q][jj];
        re[q] += a.re * b.re - a.im * b.im;
        im[q] += a.re * b.im + a.im * b.re;
      }
  }
#pragma unroll
  for (int q = 0; q < kMaxGroup; ++q)
    if (q < n) {
      const R sr = wave_sum(re[q]), si = wave_sum(im[q]);
      if (lane == 0) {
        cplx<R> o;
        o.re = sr;
        o.im = si;
        ys[q][i] = o;
      }
    }
}

// Every group has one member: lean kernel (no per-member arrays, full
// occupancy), four independent loads in flight per lane.
template <typename R>
__global__ __launch_bounds__(256) void k_dense_gemv_desc1(const SysDesc* __restrict__ sd,
                                                          const GemvGroup* __restrict__ groups,
                                                          const RowBlock* __restrict__ map, int which,
                                                          int j, unsigned long long* ctr) {
  const RowBlock rb = map[blockIdx.x];
  const SysDesc D = sd[groups[rb.group].sys[0]];
  if (which == 0 ? !D.sysi[1] : !D.sysi[0]) return;
  const int lane = threadIdx.x & 63;
  const int i = rb.row0 + (threadIdx.x >> 6);
  const int M = D.M;
  if (ctr && threadIdx.x == 0 && rb.row0 == 0) {
    const unsigned long long MM = (unsigned long long)M;
    atomicAdd(ctr, (MM * MM + 2 * MM) * sizeof(cplx<R>));
  }
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
void launch_dense_gemv_desc(const SysDesc* sd, const GemvGroup* groups, const RowBlock* map,
                            int nblocks, int which, int j, bool grouped, unsigned long long* ctr,
                            hipStream_t s) {
  if (grouped)
    hipLaunchKernelGGL((k_dense_gemv_desc<R>), dim3(nblocks), dim3(256), 0, s, sd, groups, map, which, j, ctr);
  else
    hipLaunchKernelGGL((k_dense_gemv_desc1<R>), dim3(nblocks), dim3(256), 0, s, sd, groups, map, which, j, ctr);
  CQM_HIP(hipGetLastError());
}
template void launch_dense_gemv_desc<float>(const SysDesc*, const GemvGroup*, const RowBlock*, int, int,
                                            int, bool, unsigned long long*, hipStream_t);
template void launch_dense_gemv_desc<double>(const SysDesc*, const GemvGroup*, const RowBlock*, int, int,
                                             int, bool, unsigned long long*, hipStream_t);

template void launch_dense_gemv<float>(const cf32*, int, int, const cf32*, int64_t, cf32*, int64_t,
                                       const int*, hipStream_t);
template void launch_dense_gemv<double>(const cf64*, int, int, const cf64*, int64_t, cf64*,
                                        int64_t, const int*, hipStream_t);

}  // namespace cqm
