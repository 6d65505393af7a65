// Batched restarted GMRES: one workgroup per frequency system, all systems
// advanced by the same launches.  Each restart cycle begins from the FP64 true
// residual r = ghat - V x (computed by the caller), so restarts double as
// iterative-refinement steps: the Krylov basis may be FP32 while x and r stay
// FP64.  Orthogonalisation is classical Gram-Schmidt applied twice; the
// Hessenberg matrix, Givens rotations and the residual estimate are FP64.
// Per-system status lives on the device, so a cycle needs no host round trip.
#include "device_util.h"

namespace cqm {

namespace {
constexpr int kChunk = 16;  // inner products per pass over w (one pass for j < 16)
constexpr int kMaxM = 64;   // largest supported restart length
constexpr double kFloorTol = 1e-13;  // stagnation below this counts as converged
}  // namespace

// sysd per system (8 doubles): 0 beta, 1 cycle tolerance, 2 ||ghat||,
// 3 last true residual norm, 4 non-finite flag.  sysi (kSysiStride ints):
// 0 system active, 1 cycle active, 2 Arnoldi steps in cycle, 3 total steps.
// Every kernel takes the system descriptors; workgroup k serves system k, so
// systems of different lengths and problems share the launches.
__global__ __launch_bounds__(256) void k_gmres_init(const SysDesc* __restrict__ sd) {
  __shared__ double red[16];
  const SysDesc D = sd[blockIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < D.M; i += 256) {
    const cf64 v = D.ghat[i];
    acc += v.re * v.re + v.im * v.im;
    D.x[i] = cf64{0.0, 0.0};
    D.r[i] = v;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 8; ++k) D.sysd[k] = 0.0;
    D.sysd[2] = sqrt(acc);
    D.sysd[3] = D.sysd[2];
    D.sysi[0] = 1;
    D.sysi[1] = 0;
    D.sysi[2] = 0;
    D.sysi[3] = 0;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cycle_start(const SysDesc* __restrict__ sd, double outer_tol,
                                                     double inner_tol) {
  __shared__ double red[16];
  const SysDesc D = sd[blockIdx.x];
  int* st = D.sysi;
  double* d = D.sysd;
  if (!st[0]) return;
  const int M = D.M, m = D.m;
  const cf64* rl = D.r;
  double acc = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) acc += rl[i].re * rl[i].re + rl[i].im * rl[i].im;
  const double rn = sqrt(block_sum(acc, red));
  const double bn = d[2];
  if (!isfinite(rn)) {
    if (threadIdx.x == 0) {
      d[4] = 1.0;
      st[0] = 0;
      st[1] = 0;
    }
    return;
  }
  // converged, or stagnated at the FP64 floor: a restart that no longer halves
  // a true residual already below kFloorTol counts as converged
  const double prev = d[3];
  if (rn <= outer_tol * bn || rn == 0.0 || (rn > 0.5 * prev && rn <= kFloorTol * bn)) {
    if (threadIdx.x == 0) {
      d[3] = rn;
      st[0] = 0;
      st[1] = 0;
    }
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d[0] = rn;
    d[1] = fmax(inner_tol * rn, 0.5 * outer_tol * bn);
    d[3] = rn;
    st[1] = 1;
    st[2] = 0;
  }
  for (int k = threadIdx.x; k <= m; k += 256) D.g[k] = cf64{k == 0 ? rn : 0.0, 0.0};
  cplx<R>* v0 = (cplx<R>*)D.basis;
  const double inv = 1.0 / rn;
  for (int i = threadIdx.x; i < M; i += 256) {
    cplx<R> o;
    o.re = (R)(rl[i].re * inv);
    o.im = (R)(rl[i].im * inv);
    v0[i] = o;
  }
}

// r <- ghat - r for open systems (r holds V x on entry).
__global__ __launch_bounds__(256) void k_residual_combine(const SysDesc* __restrict__ sd) {
  const SysDesc D = sd[blockIdx.x];
  if (!D.sysi[0]) return;
  for (int i = threadIdx.x; i < D.M; i += 256)
    D.r[i] = cf64{D.ghat[i].re - D.r[i].re, D.ghat[i].im - D.r[i].im};
}

// status of every system into one array (one host copy per check)
__global__ void k_gather_status(const SysDesc* __restrict__ sd, int n, int* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int* st = sd[k].sysi;
  for (int q = 0; q < kSysiStride; ++q) out[k * kSysiStride + q] = st[q];
}

// One Arnoldi step of every open system.  Classical Gram-Schmidt with the
// DGKS criterion: a second pass is made only if the first one removed more
// than about 30% of the norm of w (||w'||^2 < 0.49 ||w||^2, with ||w'||^2
// accumulated while w is updated).  BS threads per system.
template <typename R, int BS>
__global__ __launch_bounds__(BS) void k_arnoldi(const SysDesc* __restrict__ sd, int j) {
  constexpr int NW = BS / 64;
  __shared__ double red[NW * (2 * kChunk + 1)];
  __shared__ cf64 coef[kMaxM + 1];
  __shared__ cf64 hacc[kMaxM + 2];
  __shared__ double rc_s[kMaxM];  // previous rotations, prefetched for thread 0
  __shared__ cf64 rs_s[kMaxM];
  __shared__ cf64 g_j;
  const SysDesc D = sd[blockIdx.x];
  int* st = D.sysi;
  if (!st[1]) return;
  const int M = D.M, m = D.m;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  cplx<R>* V = (cplx<R>*)D.basis;
  cplx<R>* w = V + (int64_t)(j + 1) * M;
  for (int k = tid; k <= j + 1; k += BS) hacc[k] = cf64{0.0, 0.0};
  for (int k = tid; k < j; k += BS) {
    rc_s[k] = D.cs[k];
    rs_s[k] = D.sn[k];
  }
  if (tid == 0) g_j = D.g[j];
  double nrm2 = 0.0;  // ||w||^2 after the last update
  for (int pass = 0; pass < 2; ++pass) {
    double w2 = 0.0;  // ||w||^2 before this pass
    for (int kc = 0; kc <= j; kc += kChunk) {
      double ar[kChunk], ai[kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) ar[u] = ai[u] = 0.0;
      double ww = 0.0;
      for (int i = tid; i < M; i += BS) {
        const cplx<R> x = w[i];
        if (kc == 0) ww += (double)x.re * x.re + (double)x.im * x.im;
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
          if (kc + u <= j) {
            const cplx<R> v = V[(int64_t)(kc + u) * M + i];
            ar[u] += (double)v.re * x.re + (double)v.im * x.im;
            ai[u] += (double)v.re * x.im - (double)v.im * x.re;
          }
      }
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        ar[u] = wave_sum(ar[u]);
        ai[u] = wave_sum(ai[u]);
      }
      ww = wave_sum(ww);
      __syncthreads();
      if (lane == 0) {
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          red[(wv * kChunk + u) * 2] = ar[u];
          red[(wv * kChunk + u) * 2 + 1] = ai[u];
        }
        red[NW * 2 * kChunk + wv] = ww;
      }
      __syncthreads();
      if (tid < kChunk && kc + tid <= j) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < NW; ++q) {
          sr += red[(q * kChunk + tid) * 2];
          si += red[(q * kChunk + tid) * 2 + 1];
        }
        coef[kc + tid] = cf64{sr, si};
      }
      if (kc == 0) {
        double t = 0.0;
        for (int q = 0; q < NW; ++q) t += red[NW * 2 * kChunk + q];
        w2 = t;
      }
    }
    __syncthreads();
    // w <- w - sum_k c_k v_k, accumulating ||w||^2 of the result
    double acc = 0.0;
    for (int i = tid; i < M; i += BS) {
      const cplx<R> x = w[i];
      double re = x.re, im = x.im;
      for (int k = 0; k <= j; ++k) {
        const cplx<R> v = V[(int64_t)k * M + i];
        const cf64 c = coef[k];
        re -= c.re * v.re - c.im * v.im;
        im -= c.re * v.im + c.im * v.re;
      }
      cplx<R> o;
      o.re = (R)re;
      o.im = (R)im;
      w[i] = o;
      acc += (double)o.re * o.re + (double)o.im * o.im;
    }
    for (int k = tid; k <= j; k += BS) {
      hacc[k].re += coef[k].re;
      hacc[k].im += coef[k].im;
    }
    acc = wave_sum(acc);
    __syncthreads();
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    nrm2 = 0.0;
    for (int q = 0; q < NW; ++q) nrm2 += red[q];
    if (nrm2 >= 0.49 * w2) break;  // block-uniform decision
    __syncthreads();
  }
  const double nr = sqrt(nrm2);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = tid; i < M; i += BS) {
    cplx<R> o = w[i];
    o.re = (R)(o.re * inv);
    o.im = (R)(o.im * inv);
    w[i] = o;
  }
  if (tid == 0) {
    cf64* Hc = D.H + (int64_t)(m + 1) * j;
    double* csl = D.cs;
    cf64* snl = D.sn;
    cf64* gl = D.g;
    cf64 h[kMaxM + 2];
    for (int k = 0; k <= j; ++k) h[k] = hacc[k];
    h[j + 1] = cf64{nr, 0.0};
    // previous rotations: (h_k, h_k+1) <- (c h_k + s h_k+1, -conj(s) h_k + c h_k+1)
    for (int k = 0; k < j; ++k) {
      const double c = rc_s[k];
      const cf64 s = rs_s[k], a = h[k], b = h[k + 1];
      h[k] = cf64{c * a.re + s.re * b.re - s.im * b.im, c * a.im + s.re * b.im + s.im * b.re};
      h[k + 1] = cf64{-(s.re * a.re + s.im * a.im) + c * b.re, -(s.re * a.im - s.im * a.re) + c * b.im};
    }
    // new rotation zeroing h_{j+1}
    const cf64 a = h[j];
    const double bb = h[j + 1].re;  // real, >= 0
    const double na = sqrt(a.re * a.re + a.im * a.im);
    double c;
    cf64 s, rr;
    if (na == 0.0) {
      c = 0.0;
      s = cf64{1.0, 0.0};
      rr = cf64{bb, 0.0};
    } else {
      const double t = sqrt(na * na + bb * bb);
      const cf64 ph{a.re / na, a.im / na};
      c = na / t;
      s = cf64{ph.re * bb / t, ph.im * bb / t};
      rr = cf64{ph.re * t, ph.im * t};
    }
    csl[j] = c;
    snl[j] = s;
    h[j] = rr;
    for (int k = 0; k <= j; ++k) Hc[k] = h[k];
    const cf64 gj = g_j;
    gl[j + 1] = cf64{-(s.re * gj.re + s.im * gj.im), -(s.re * gj.im - s.im * gj.re)};
    gl[j] = cf64{c * gj.re, c * gj.im};
    const double res = sqrt(gl[j + 1].re * gl[j + 1].re + gl[j + 1].im * gl[j + 1].im);
    st[2] = j + 1;
    st[3] += 1;
    if (!(res > D.sysd[1]) || j + 1 >= m || nr == 0.0) st[1] = 0;
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cycle_finish(const SysDesc* __restrict__ sd) {
  __shared__ cf64 y[kMaxM];
  const SysDesc D = sd[blockIdx.x];
  const int* st = D.sysi;
  if (!st[0]) return;
  const int k = st[2];
  if (k == 0) return;
  const int M = D.M, m = D.m;
  const cf64* Hl = D.H;
  const cf64* gl = D.g;
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double re = gl[i].re, im = gl[i].im;
      for (int t = i + 1; t < k; ++t) {
        const cf64 a = Hl[(int64_t)(m + 1) * t + i];
        re -= a.re * y[t].re - a.im * y[t].im;
        im -= a.re * y[t].im + a.im * y[t].re;
      }
      const cf64 d = Hl[(int64_t)(m + 1) * i + i];
      const double dn = d.re * d.re + d.im * d.im;
      y[i] = cf64{(re * d.re + im * d.im) / dn, (im * d.re - re * d.im) / dn};
    }
  }
  __syncthreads();
  const cplx<R>* V = (const cplx<R>*)D.basis;
  cf64* xl = D.x;
  for (int i = threadIdx.x; i < M; i += 256) {
    double re = xl[i].re, im = xl[i].im;
    for (int t = 0; t < k; ++t) {
      const cplx<R> v = V[(int64_t)t * M + i];
      re += y[t].re * v.re - y[t].im * v.im;
      im += y[t].re * v.im + y[t].im * v.re;
    }
    xl[i] = cf64{re, im};
  }
}

void launch_gmres_init(const SysDesc* sd, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_init, dim3(n), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}
void launch_residual_combine(const SysDesc* sd, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_residual_combine, dim3(n), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}
void launch_gather_status(const SysDesc* sd, int n, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_status, dim3((n + 255) / 256), dim3(256), 0, s, sd, n, out);
  CQM_HIP(hipGetLastError());
}
template <typename R>
void launch_cycle_start(const SysDesc* sd, int n, double outer_tol, double inner_tol, hipStream_t s) {
  hipLaunchKernelGGL((k_cycle_start<R>), dim3(n), dim3(256), 0, s, sd, outer_tol, inner_tol);
  CQM_HIP(hipGetLastError());
}
// Threads per system: latency of the block reductions dominates for short
// vectors, memory parallelism for long ones.
template <typename R> void launch_arnoldi(const SysDesc* sd, int n, int maxM, int j, hipStream_t s) {
  if (maxM < 3072)
    hipLaunchKernelGGL((k_arnoldi<R, 256>), dim3(n), dim3(256), 0, s, sd, j);
  else
    hipLaunchKernelGGL((k_arnoldi<R, 1024>), dim3(n), dim3(1024), 0, s, sd, j);
  CQM_HIP(hipGetLastError());
}
template <typename R> void launch_cycle_finish(const SysDesc* sd, int n, hipStream_t s) {
  hipLaunchKernelGGL((k_cycle_finish<R>), dim3(n), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}

template void launch_cycle_start<float>(const SysDesc*, int, double, double, hipStream_t);
template void launch_cycle_start<double>(const SysDesc*, int, double, double, hipStream_t);
template void launch_arnoldi<float>(const SysDesc*, int, int, int, hipStream_t);
template void launch_arnoldi<double>(const SysDesc*, int, int, int, hipStream_t);
template void launch_cycle_finish<float>(const SysDesc*, int, hipStream_t);
template void launch_cycle_finish<double>(const SysDesc*, int, hipStream_t);

}  // namespace cqm
