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

// New Hessenberg column h[0..j+1] of system D (h[j+1] = ||w|| real): the
// previous rotations are applied, a new one zeroes h[j+1], the column and
// the residual estimate |g[j+1]| are stored, and the cycle closes when that
// estimate meets the cycle tolerance, the basis is full or w vanished.
// Called by one thread; rc, rs hold the previous rotations, gj = g[j].
__device__ void hessenberg_column(const SysDesc& D, int j, cf64* h, const double* rc,
                                  const cf64* rs, cf64 gj, double nr) {
  const int m = D.m;
  cf64* Hc = D.H + (int64_t)(m + 1) * j;
  // previous rotations: (h_k, h_k+1) <- (c h_k + s h_k+1, -conj(s) h_k + c h_k+1)
  for (int k = 0; k < j; ++k) {
    const double c = rc[k];
    const cf64 s = rs[k], a = h[k], b = h[k + 1];
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
  D.cs[j] = c;
  D.sn[j] = s;
  h[j] = rr;
  for (int k = 0; k <= j; ++k) Hc[k] = h[k];
  cf64* gl = D.g;
  gl[j + 1] = cf64{-(s.re * gj.re + s.im * gj.im), -(s.re * gj.im - s.im * gj.re)};
  gl[j] = cf64{c * gj.re, c * gj.im};
  const double res = sqrt(gl[j + 1].re * gl[j + 1].re + gl[j + 1].im * gl[j + 1].im);
  int* st = D.sysi;
  st[2] = j + 1;
  st[3] += 1;
  if (!(res > D.sysd[1]) || j + 1 >= m || nr == 0.0) st[1] = 0;
}

// acc += sign * sum_{k < n} c_k v_k[i] for basis vectors v_k = V + k M
// (c_k in LDS): the loads of a chunk of kU vectors are issued together so
// that a thread keeps kU loads in flight instead of one.
template <typename R, int kU>
__device__ __forceinline__ void basis_combine(const cplx<R>* __restrict__ V, int64_t M, int i,
                                              const cf64* c, int n, double sign, double& re,
                                              double& im) {
  for (int kc = 0; kc < n; kc += kU) {
    // clamped (in-bounds) loads, all in flight together; terms beyond n are
    // dropped by a zero coefficient
    cplx<R> v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) v[u] = V[(int64_t)min(kc + u, n - 1) * M + i];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool in = kc + u < n;
      const cf64 cu = c[min(kc + u, n - 1)];
      const cf64 a{in ? sign * cu.re : 0.0, in ? sign * cu.im : 0.0};
      re += a.re * v[u].re - a.im * v[u].im;
      im += a.re * v[u].im + a.im * v[u].re;
    }
  }
}


// One Arnoldi step of every open system.  Classical Gram-Schmidt with the
// DGKS criterion: a second pass is made only if the first one removed more
// than about 30% of the norm of w (||w'||^2 < 0.49 ||w||^2, with ||w'||^2
// accumulated while w is updated).  BS threads per system.
template <typename R, int BS>
__global__ __launch_bounds__(BS) void k_arnoldi(const SysDesc* __restrict__ sd, int j,
                                                unsigned long long* ctr) {
  // inner products per pass over w: all of them for j < 32 with 4 waves,
  // half as many with 16 waves (register budget)
  constexpr int kChunk = BS <= 256 ? 32 : 8;
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
      // entries 0..kChunk-1: real parts, kChunk..2kChunk-1: imaginary parts
      double a2[2 * kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        a2[u] = ar[u];
        a2[kChunk + u] = ai[u];
      }
      wave_reduce_scatter<2 * kChunk, 32>(a2, lane);
      ww = wave_sum(ww);
      constexpr int kSh = 6 - (kChunk == 32 ? 6 : kChunk == 16 ? 5 : kChunk == 8 ? 4 : 3);
      __syncthreads();
      if ((lane & ((1 << kSh) - 1)) == 0) red[wv * 2 * kChunk + (lane >> kSh)] = a2[0];
      if (lane == 0) red[NW * 2 * kChunk + wv] = ww;
      __syncthreads();
      if (tid < kChunk && kc + tid <= j) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < NW; ++q) {
          sr += red[q * 2 * kChunk + tid];
          si += red[q * 2 * kChunk + kChunk + tid];
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
      basis_combine<R, 16>(V, M, i, coef, j + 1, -1.0, re, im);
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
    if (ctr && tid == 0) {
      // one Gram-Schmidt pass: read v_0..v_j and w (inner products), read
      // v_0..v_j and w and write w (update)
      atomicAdd(ctr, (unsigned long long)(2 * (j + 1) + 3) * M * sizeof(cplx<R>));
    }
    if (nrm2 >= 0.49 * w2) break;  // block-uniform decision
    __syncthreads();
  }
  if (ctr && tid == 0) atomicAdd(ctr, (unsigned long long)2 * M * sizeof(cplx<R>));  // normalisation
  const double nr = sqrt(nrm2);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int i = tid; i < M; i += BS) {
    cplx<R> o = w[i];
    o.re = (R)(o.re * inv);
    o.im = (R)(o.im * inv);
    w[i] = o;
  }
  __shared__ cf64 h[kMaxM + 2];
  if (tid == 0) {
    for (int k = 0; k <= j; ++k) h[k] = hacc[k];
    h[j + 1] = cf64{nr, 0.0};
    hessenberg_column(D, j, h, rc_s, rs_s, g_j, nr);
  }
}

// ------------------------------------------------------------------
// The same Arnoldi step split over S = ceil(M / kArnRows) workgroups per
// system, one row per thread, for batches with fewer systems than compute
// units.  Three launches per step:
//   dots    c = V^H w and ||w||^2, per slice;
//   update  w' = w - V c, then c' = V^H w' and ||w'||^2, per slice;
//   finish  DGKS test; if a second pass is needed w'' = w' - V c' with
//           ||w''||^2 = ||w'||^2 - ||c'||^2 (V orthonormal); scale by 1/||w''||;
//           slice 0 forms the Hessenberg column c + c' and the rotation.
// Partial sums live in D.part, per slice: P1 (m+1 cf64), P2 (m+1 cf64),
// ||w||^2, ||w'||^2.  Every workgroup reduces them over the slices in the
// same order, so all workgroups of a system take identical decisions.
__device__ __forceinline__ int arn_stride(int m) { return 4 * (m + 1) + 2; }

// out[k] (k <= j) = sum over this slice of conj(v_k[i]) x_i (x_i = 0 and no
// loads where !valid); kC inner products per reduction round.
template <typename R, int kC>
__device__ __forceinline__ void slice_dots(const cplx<R>* __restrict__ V, int64_t M, int i, bool valid,
                           cplx<R> x, int j, cf64* out, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kArnRows / 64;
  // loads use clamped (in-bounds) indices and are masked afterwards, so all
  // kC of them are in flight together
  const int ic = valid ? i : (int)M - 1;
  for (int kc = 0; kc <= j; kc += kC) {
    cplx<R> v[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) v[u] = V[(int64_t)min(kc + u, j) * M + ic];
    double a[2 * kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const bool in = valid && kc + u <= j;
      const double vr = in ? (double)v[u].re : 0.0, vi = in ? (double)v[u].im : 0.0;
      a[u] = vr * x.re + vi * x.im;
      a[kC + u] = vr * x.im - vi * x.re;
    }
    wave_reduce_scatter<2 * kC, 32>(a, lane);
    constexpr int kSh = kC == 32 ? 0 : kC == 16 ? 1 : 2;
    __syncthreads();
    if ((lane & ((1 << kSh) - 1)) == 0) red[wv * 2 * kC + (lane >> kSh)] = a[0];
    __syncthreads();
    if (tid < kC && kc + tid <= j) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) {
        sr += red[q * 2 * kC + tid];
        si += red[q * 2 * kC + kC + tid];
      }
      out[kc + tid] = cf64{sr, si};
    }
  }
}

// inner products per reduction round (register budget: 2 kC doubles and kC
// loaded basis entries per thread)
template <typename R> struct ArnChunk { static constexpr int v = 16; };

template <typename R>
__global__ __launch_bounds__(kArnRows) void k_arn_dots(const SysDesc* __restrict__ sd, int j,
                                                      int fused, unsigned long long* ctr) {
  constexpr int kC = ArnChunk<R>::v;
  __shared__ double red[(kArnRows / 64) * 2 * kC];
  const SysDesc D = sd[blockIdx.y];
  if (!D.sysi[1]) return;
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  if (s * kArnRows >= M) return;
  const int i = s * kArnRows + threadIdx.x;
  const bool valid = i < M;
  cplx<R>* V = (cplx<R>*)D.basis;
  cplx<R> x;
  x.re = R(0);
  x.im = R(0);
  if (valid) {
    if (fused && D.symp) {
      // w = A v_j of a stored operator: sum its tile partials here
      x = sym_row_sum<R>((const cplx<R>*)D.symp, M, i);
      V[(int64_t)(j + 1) * M + i] = x;
    } else {
      x = V[(int64_t)(j + 1) * M + i];
    }
  }
  double* P = D.part + (int64_t)s * arn_stride(m);
  slice_dots<R, kC>(V, M, i, valid, x, j, reinterpret_cast<cf64*>(P), red);
  const double nn = block_sum((double)x.re * x.re + (double)x.im * x.im, red);
  if (threadIdx.x == 0) {
    P[4 * (m + 1)] = nn;
    if (ctr) {
      const unsigned long long rows = min(kArnRows, M - s * kArnRows);
      atomicAdd(ctr, rows * (j + 2) * sizeof(cplx<R>));
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kArnRows) void k_arn_update(const SysDesc* __restrict__ sd, int j,
                                                        unsigned long long* ctr) {
  constexpr int kC = ArnChunk<R>::v;
  __shared__ double red[(kArnRows / 64) * 2 * kC];
  __shared__ cf64 coef[kMaxM + 1];
  const SysDesc D = sd[blockIdx.y];
  if (!D.sysi[1]) return;
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  if (s * kArnRows >= M) return;
  const int S = (M + kArnRows - 1) / kArnRows;
  const int str = arn_stride(m);
  for (int k = threadIdx.x; k <= j; k += kArnRows)
    coef[k] = cf64{slot_sum(D.part + 2 * k, S, str), slot_sum(D.part + 2 * k + 1, S, str)};
  __syncthreads();
  const int i = s * kArnRows + threadIdx.x;
  const bool valid = i < M;
  cplx<R>* V = (cplx<R>*)D.basis;
  cplx<R> x;
  x.re = R(0);
  x.im = R(0);
  if (valid) {
    cplx<R>* w = V + (int64_t)(j + 1) * M;
    const cplx<R> x0 = w[i];
    double re = x0.re, im = x0.im;
    basis_combine<R, 16>(V, M, i, coef, j + 1, -1.0, re, im);
    x.re = (R)re;
    x.im = (R)im;
    w[i] = x;
  }
  double* P = D.part + (int64_t)s * str;
  slice_dots<R, kC>(V, M, i, valid, x, j, reinterpret_cast<cf64*>(P + 2 * (m + 1)), red);
  const double nn = block_sum((double)x.re * x.re + (double)x.im * x.im, red);
  if (threadIdx.x == 0) {
    P[4 * (m + 1) + 1] = nn;
    if (ctr) {
      const unsigned long long rows = min(kArnRows, M - s * kArnRows);
      atomicAdd(ctr, rows * (j + 3) * sizeof(cplx<R>));
    }
  }
}

template <typename R>
__global__ __launch_bounds__(kArnRows) void k_arn_finish(const SysDesc* __restrict__ sd, int j,
                                                        unsigned long long* ctr) {
  __shared__ cf64 c2[kMaxM + 1];
  __shared__ cf64 h[kMaxM + 2];
  __shared__ double rc_s[kMaxM];
  __shared__ cf64 rs_s[kMaxM];
  __shared__ double nsh[2];
  __shared__ int second_s;
  const SysDesc D = sd[blockIdx.y];
  if (!D.sysi[1]) return;
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  if (s * kArnRows >= M) return;
  const int S = (M + kArnRows - 1) / kArnRows;
  const int str = arn_stride(m);
  const int tid = threadIdx.x;
  if (tid == 0) {
    const double n0 = slot_sum(D.part + 4 * (m + 1), S, str);
    const double n1 = slot_sum(D.part + 4 * (m + 1) + 1, S, str);
    nsh[0] = n0;
    nsh[1] = n1;
    second_s = n1 < 0.49 * n0;
  }
  __syncthreads();
  const bool second = second_s != 0;
  for (int k = tid; k <= j; k += kArnRows) {
    const double* P = D.part + 2 * (m + 1) + 2 * k;
    c2[k] = second ? cf64{slot_sum(P, S, str), slot_sum(P + 1, S, str)} : cf64{0.0, 0.0};
  }
  __syncthreads();
  if (tid == 0) {
    double n2 = nsh[1];
    if (second) {
      for (int k = 0; k <= j; ++k) n2 -= c2[k].re * c2[k].re + c2[k].im * c2[k].im;
      n2 = fmax(n2, 0.0);
    }
    nsh[0] = sqrt(n2);
  }
  __syncthreads();
  const double nr = nsh[0];
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  const int i = s * kArnRows + tid;
  cplx<R>* V = (cplx<R>*)D.basis;
  if (i < M) {
    cplx<R>* w = V + (int64_t)(j + 1) * M;
    const cplx<R> x0 = w[i];
    double re = x0.re, im = x0.im;
    if (second) basis_combine<R, 16>(V, M, i, c2, j + 1, -1.0, re, im);
    cplx<R> o;
    o.re = (R)(re * inv);
    o.im = (R)(im * inv);
    w[i] = o;
  }
  if (ctr && tid == 0) {
    const unsigned long long rows = min(kArnRows, M - s * kArnRows);
    atomicAdd(ctr, rows * (second ? j + 3 : 2) * sizeof(cplx<R>));
  }
  if (s != 0) return;
  for (int k = tid; k <= j; k += kArnRows)
    h[k] = cf64{slot_sum(D.part + 2 * k, S, str) + c2[k].re,
                slot_sum(D.part + 2 * k + 1, S, str) + c2[k].im};
  for (int k = tid; k < j; k += kArnRows) {
    rc_s[k] = D.cs[k];
    rs_s[k] = D.sn[k];
  }
  __syncthreads();
  if (tid == 0) {
    h[j + 1] = cf64{nr, 0.0};
    hessenberg_column(D, j, h, rc_s, rs_s, D.g[j], nr);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cycle_finish(const SysDesc* __restrict__ sd) {
  __shared__ cf64 y[kMaxM];
  __shared__ cf64 Hs[kMaxM * (kMaxM + 1) / 2];  // upper triangle, column by column
  const SysDesc D = sd[blockIdx.x];
  const int* st = D.sysi;
  if (!st[0]) return;
  const int k = st[2];
  if (k == 0) return;
  const int M = D.M, m = D.m;
  const cf64* Hl = D.H;
  const cf64* gl = D.g;
  // column t of the triangular factor holds rows 0..t: offset t (t+1) / 2
  for (int e = threadIdx.x; e < k * (k + 1) / 2; e += 256) {
    int t = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > e) --t;
    while ((t + 1) * (t + 2) / 2 <= e) ++t;
    const int r = e - t * (t + 1) / 2;
    Hs[e] = Hl[(int64_t)(m + 1) * t + r];
  }
  if (threadIdx.x < k) y[threadIdx.x] = gl[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double re = y[i].re, im = y[i].im;
      for (int t = i + 1; t < k; ++t) {
        const cf64 a = Hs[t * (t + 1) / 2 + i];
        re -= a.re * y[t].re - a.im * y[t].im;
        im -= a.re * y[t].im + a.im * y[t].re;
      }
      const cf64 d = Hs[i * (i + 1) / 2 + i];
      const double dn = d.re * d.re + d.im * d.im;
      y[i] = cf64{(re * d.re + im * d.im) / dn, (im * d.re - re * d.im) / dn};
    }
  }
  __syncthreads();
  const cplx<R>* V = (const cplx<R>*)D.basis;
  cf64* xl = D.x;
  for (int i = threadIdx.x; i < M; i += 256) {
    double re = xl[i].re, im = xl[i].im;
    basis_combine<R, 16>(V, M, i, y, k, 1.0, re, im);
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
// One workgroup per system (threads per system: latency of the block
// reductions dominates for short vectors, memory parallelism for long ones),
// or the three-launch split over row slices.
template <typename R>
void launch_arnoldi(const SysDesc* sd, int n, int maxM, int j, bool split, bool fused,
                    unsigned long long* ctr, hipStream_t s) {
  if (split) {
    const dim3 grid((maxM + kArnRows - 1) / kArnRows, n);
    hipLaunchKernelGGL((k_arn_dots<R>), grid, dim3(kArnRows), 0, s, sd, j, fused ? 1 : 0, ctr);
    hipLaunchKernelGGL((k_arn_update<R>), grid, dim3(kArnRows), 0, s, sd, j, ctr);
    hipLaunchKernelGGL((k_arn_finish<R>), grid, dim3(kArnRows), 0, s, sd, j, ctr);
  } else if (maxM < 3072) {
    hipLaunchKernelGGL((k_arnoldi<R, 256>), dim3(n), dim3(256), 0, s, sd, j, ctr);
  } else {
    hipLaunchKernelGGL((k_arnoldi<R, 1024>), dim3(n), dim3(1024), 0, s, sd, j, ctr);
  }
  CQM_HIP(hipGetLastError());
}
template <typename R> void launch_cycle_finish(const SysDesc* sd, int n, hipStream_t s) {
  hipLaunchKernelGGL((k_cycle_finish<R>), dim3(n), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}

template void launch_cycle_start<float>(const SysDesc*, int, double, double, hipStream_t);
template void launch_cycle_start<double>(const SysDesc*, int, double, double, hipStream_t);
template void launch_arnoldi<float>(const SysDesc*, int, int, int, bool, bool,
                                    unsigned long long*, hipStream_t);
template void launch_arnoldi<double>(const SysDesc*, int, int, int, bool, bool,
                                     unsigned long long*, hipStream_t);
template void launch_cycle_finish<float>(const SysDesc*, int, hipStream_t);
template void launch_cycle_finish<double>(const SysDesc*, int, hipStream_t);

}  // namespace cqm
