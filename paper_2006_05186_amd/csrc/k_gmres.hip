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
// 0 system active, 1 cycle active, 2 Arnoldi steps in cycle, 3 total steps,
// 4 the residual closing this cycle is formed in double-double (set per
// system at the cycle's start, so a system's arithmetic never depends on
// the others it shares a batch with).
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
    D.sysi[4] = 0;
  }
}

// relax > 0 (inexact refinement): once a cycle has reduced the true
// residual by q = rn / previous, the next cycle's inner target is relaxed to
// relax * q of its start (at most 1e-3, never tighter than inner_tol): when
// the inner operator only approximates the one of the residual, each cycle
// gains about q, and solving the inner system further gains nothing.
template <typename R>
__global__ __launch_bounds__(256) void k_cycle_start(const SysDesc* __restrict__ sd, double outer_tol,
                                                     double inner_tol, double relax) {
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
    double itol = inner_tol;
    if (relax > 0.0 && rn < prev) itol = fmax(inner_tol, fmin(relax * rn / prev, 1e-3));
    d[0] = rn;
    d[1] = fmax(itol * rn, 0.5 * outer_tol * bn);
    d[3] = rn;
    st[1] = 1;
    st[2] = 0;
    // double-double closing residual: FP64 inner cycles, and FP32 ones whose
    // residual is already below 1e-6 (before that, FP64 rounding of V x is
    // far below the cycle's gain and the next cycle corrects it)
    st[4] = (sizeof(R) == 8 || rn <= 1e-6 * bn) ? 1 : 0;
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
// Stored-operator systems (symp set) have theirs formed by the product's
// reduction already.
__global__ __launch_bounds__(256) void k_residual_combine(const SysDesc* __restrict__ sd) {
  const SysDesc D = sd[blockIdx.x];
  if (!D.sysi[0] || D.symp) return;
  for (int i = threadIdx.x; i < D.M; i += 256)
    D.r[i] = cf64{D.ghat[i].re - D.r[i].re, D.ghat[i].im - D.r[i].im};
}

// status of every system into one array, written straight into pinned host
// memory (made visible to the host before the kernel ends)
__global__ void k_gather_diag(const SysDesc* __restrict__ sd, int n, int* __restrict__ flags,
                              double* __restrict__ norms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const SysDesc& D = sd[k];
  for (int q = 0; q < kSysiStride; ++q) flags[k * kSysiStride + q] = D.sysi[q];
  for (int q = 0; q < 3; ++q) norms[3 * k + q] = D.sysd[2 + q];
  __threadfence_system();
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
  // the running entry h[k] is carried in registers: only it depends on the
  // previous rotation, the loads of rc, rs and h[k+1] do not
  if (j > 0) {
    cf64 a = h[0];
#pragma unroll 4
    for (int k = 0; k < j; ++k) {
      const double c = rc[k];
      const cf64 s = rs[k], b = h[k + 1];
      h[k] = cf64{c * a.re + s.re * b.re - s.im * b.im, c * a.im + s.re * b.im + s.im * b.re};
      a = cf64{-(s.re * a.re + s.im * a.im) + c * b.re, -(s.re * a.im - s.im * a.re) + c * b.im};
    }
    h[j] = a;
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
  if (D.hflag) {
    // host-visible copy, read after the step's completion event
    *D.hflag = st[1];
    __threadfence_system();
  }
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


// Progress word in pinned host memory: the last kernel of Arnoldi step j
// stores j + 1 when it starts, so everything queued before it (earlier
// steps, copies) has completed.  Written whether or not a system is open.
__device__ __forceinline__ void step_progress(int* prog, int j) {
  if (prog && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    *prog = j + 1;
    __threadfence_system();
  }
}

// One Arnoldi step of every open system.  Classical Gram-Schmidt with the
// DGKS criterion: a second pass is made only if the first one removed more
// than about 30% of the norm of w (||w'||^2 < 0.49 ||w||^2, with ||w'||^2
// accumulated while w is updated).  BS threads per system.
template <typename R, int BS>
__global__ __launch_bounds__(BS) void k_arnoldi(const SysDesc* __restrict__ sd, int j,
                                                unsigned long long* ctr, int* prog) {
  step_progress(prog, j);
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
  const int M = D.M;
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
        // clamped (in-bounds) loads, all in flight together
        const cplx<R> x = w[i];
        cplx<R> v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) v[u] = V[(int64_t)min(kc + u, j) * M + i];
        if (kc == 0) ww += (double)x.re * x.re + (double)x.im * x.im;
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
          if (kc + u <= j) {
            ar[u] += (double)v[u].re * x.re + (double)v[u].im * x.im;
            ai[u] += (double)v[u].re * x.im - (double)v[u].im * x.re;
          }
      }
      // entries 0..kChunk-1: real parts, kChunk..2kChunk-1: imaginary parts
      double a2[2 * kChunk];
#pragma unroll
      for (int u = 0; u < kChunk; ++u) {
        a2[u] = ar[u];
        a2[kChunk + u] = ai[u];
      }
      wave_reduce_scatter_near<2 * kChunk>(a2, lane);
      ww = wave_sum(ww);
      __syncthreads();
      if (lane < 2 * kChunk) red[wv * 2 * kChunk + scatter_entry<2 * kChunk>(lane)] = a2[0];
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

// The kernels are latency-bound (a few KB per workgroup), so each one issues
// all of its loads in one round: the open flag, the product partials or w,
// a chunk of kVC basis entries per row (held in registers and used by both
// the update and the second inner products) and the slot sums it needs.
// Closed systems and slices past the end run the same code and write
// nothing (a branch before the loads would add a dependent round trip).
// kVC, the basis vectors per register chunk, is 16 while j < 16 and 32 after
// (one chunk covers the default restart length).
constexpr int kPB = 32;  // product partials summed per round of loads

template <typename R> using gcplx = const CQM_GLOBAL cplx<R>;

template <typename R, int kVC>
__device__ __forceinline__ void load_chunk(gcplx<R>* __restrict__ V, int64_t M, int ic, int kc, int j,
                                           cplx<R> (&v)[kVC]) {
#pragma unroll
  for (int u = 0; u < kVC; ++u) v[u] = V[(int64_t)min(kc + u, j) * M + ic];
}

// Slice inner products of chunk kc with x: out[2k], out[2k+1] = re, im of
// sum_i conj(v_k[i]) x_i for kc <= k <= min(kc + kVC - 1, j); with nrm, also
// *nrm = sum_i |x_i|^2.  Written only when wr.  red: LDS, 4 (2 kVC + 1)
// doubles.
template <typename R, int kVC>
__device__ __forceinline__ void chunk_dots(const cplx<R> (&v)[kVC], cplx<R> x, bool valid, int kc,
                                           int j, bool wr, double* out, double* nrm, double* red) {
  constexpr int NW = kArnRows / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double a[2 * kVC];
#pragma unroll
  for (int u = 0; u < kVC; ++u) {
    const bool in = valid && kc + u <= j;
    const double vr = in ? (double)v[u].re : 0.0, vi = in ? (double)v[u].im : 0.0;
    a[u] = vr * x.re + vi * x.im;
    a[kVC + u] = vr * x.im - vi * x.re;
  }
  wave_reduce_scatter_near<2 * kVC>(a, lane);
  double nn = 0.0;
  if (nrm) nn = wave_sum_near(valid ? (double)x.re * x.re + (double)x.im * x.im : 0.0);
  __syncthreads();
  if (lane < 2 * kVC) red[wv * 2 * kVC + scatter_entry<2 * kVC>(lane)] = a[0];
  if (nrm && lane == 0) red[NW * 2 * kVC + wv] = nn;
  __syncthreads();
  if (wr && tid < 2 * kVC) {
    // entry t < kVC: real part of product kc + t; else imaginary part
    const int k = kc + (tid % kVC), comp = tid / kVC;
    if (k <= j) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) t += red[q * 2 * kVC + tid];
      as_global(out)[2 * k + comp] = t;
    }
  }
  if (wr && nrm && tid == 2 * kVC) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += red[NW * 2 * kVC + q];
    *as_global(nrm) = t;
  }
}

// re, im -= sum_{k in chunk} c_k v_k (c: LDS, re/im interleaved doubles).
template <typename R, int kVC>
__device__ __forceinline__ void chunk_update(const cplx<R> (&v)[kVC], int kc, int j, const double* c,
                                             double& re, double& im) {
#pragma unroll
  for (int u = 0; u < kVC; ++u) {
    const bool in = kc + u <= j;
    const int k = min(kc + u, j);
    const double cr = in ? c[2 * k] : 0.0, ci = in ? c[2 * k + 1] : 0.0;
    re -= cr * v[u].re - ci * v[u].im;
    im -= cr * v[u].im + ci * v[u].re;
  }
}

// sum_{q < S} P[q * stride] in slot order.  The first eight loads are
// straight-line code (clamped indices), so they join the caller's round of
// loads; slices beyond eight take further rounds.
__device__ __forceinline__ double slot_sum_g(const CQM_GLOBAL double* __restrict__ P, int S,
                                             int64_t stride) {
  double v[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)min(u, S - 1) * stride];
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (u < S) acc += v[u];
  for (int q0 = 8; q0 < S; q0 += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)min(q0 + u, S - 1) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (q0 + u < S) acc += v[u];
  }
  return acc;
}

template <typename R, int kVC>
__global__ __launch_bounds__(kArnRows) void k_arn_dots(const SysDesc* __restrict__ sd, int j,
                                                      int fused, unsigned long long* ctr) {
  __shared__ double red[(kArnRows / 64) * (2 * kVC + 1)];
  const SysDesc D = sd[blockIdx.y];
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  const int i = s * kArnRows + threadIdx.x;
  const bool valid = i < M;
  const int ic = valid ? i : M - 1;
  gcplx<R>* V = as_global((const cplx<R>*)D.basis);
  // w = A v_j: summed here from the tile partials of a stored operator
  const bool sum = fused && D.symp;
  const int nt = sym_blocks(M), ntB = nt * kSymB;
  gcplx<R>* Pp = as_global((const cplx<R>*)(sum ? D.symp : D.basis));
  cplx<R> pv[kPB];
  if (sum) {
#pragma unroll
    for (int u = 0; u < kPB; ++u) pv[u] = Pp[(int64_t)min(u, nt - 1) * ntB + ic];
  } else {
    pv[0] = V[(int64_t)(j + 1) * M + ic];
  }
  cplx<R> v[kVC];
  load_chunk<R, kVC>(V, M, ic, 0, j, v);
  const bool wr = *as_global(D.sysi + 1) != 0 && s * kArnRows < M;
  cplx<R> x = pv[0];
  if (sum) {
    R re = R(0), im = R(0);
#pragma unroll
    for (int u = 0; u < kPB; ++u)
      if (u < nt) {
        re += pv[u].re;
        im += pv[u].im;
      }
    for (int Y0 = kPB; Y0 < nt; Y0 += kPB) {  // meshes of more than kPB blocks
#pragma unroll
      for (int u = 0; u < kPB; ++u) pv[u] = Pp[(int64_t)min(Y0 + u, nt - 1) * ntB + ic];
#pragma unroll
      for (int u = 0; u < kPB; ++u)
        if (Y0 + u < nt) {
          re += pv[u].re;
          im += pv[u].im;
        }
    }
    x = cmake<R>(re, im);
  }
  if (!valid) x = cmake<R>(R(0), R(0));
  double* P = D.part + (int64_t)s * arn_stride(m);
  chunk_dots<R, kVC>(v, x, valid, 0, j, wr, P, P + 4 * (m + 1), red);
  for (int kc = kVC; kc <= j; kc += kVC) {
    load_chunk<R, kVC>(V, M, ic, kc, j, v);
    chunk_dots<R, kVC>(v, x, valid, kc, j, wr, P, nullptr, red);
  }
  if (!wr) return;
  if (sum && valid) as_global((cplx<R>*)D.basis)[(int64_t)(j + 1) * M + i] = x;
  if (ctr && threadIdx.x == 0) {
    // inner products: v_0 .. v_j and w; with the stored product's tile
    // partials reduced here, their nt slots per row and the sum's write
    const unsigned long long rows = min(kArnRows, M - s * kArnRows);
    atomicAdd(ctr, rows * ((j + 2) + (sum ? nt + 1 : 0)) * sizeof(cplx<R>));
  }
}

template <typename R, int kVC>
__global__ __launch_bounds__(kArnRows) void k_arn_update(const SysDesc* __restrict__ sd, int j,
                                                        unsigned long long* ctr) {
  __shared__ double red[(kArnRows / 64) * (2 * kVC + 1)];
  __shared__ double cf[2 * (kMaxM + 1)];
  const SysDesc D = sd[blockIdx.y];
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  const int S = (M + kArnRows - 1) / kArnRows;
  const int str = arn_stride(m);
  const int i = s * kArnRows + threadIdx.x;
  const bool valid = i < M;
  const int ic = valid ? i : M - 1;
  gcplx<R>* V = as_global((const cplx<R>*)D.basis);
  const cplx<R> x0 = V[(int64_t)(j + 1) * M + ic];
  cplx<R> v[kVC];
  load_chunk<R, kVC>(V, M, ic, 0, j, v);
  const CQM_GLOBAL double* part = as_global((const double*)D.part);
  {
    // coefficient entry t = threadIdx.x (clamped loads; stored if t is one)
    const int n2j = 2 * (j + 1), t = threadIdx.x;
    const double val = slot_sum_g(part + min(t, n2j - 1), S, str);
    if (t < n2j) cf[t] = val;
    for (int t2 = t + kArnRows; t2 < n2j; t2 += kArnRows) cf[t2] = slot_sum_g(part + t2, S, str);
  }
  const bool wr = *as_global(D.sysi + 1) != 0 && s * kArnRows < M;
  __syncthreads();
  // w' = w - V c
  double re = x0.re, im = x0.im;
  chunk_update<R, kVC>(v, 0, j, cf, re, im);
  for (int kc = kVC; kc <= j; kc += kVC) {
    cplx<R> u[kVC];
    load_chunk<R, kVC>(V, M, ic, kc, j, u);
    chunk_update<R, kVC>(u, kc, j, cf, re, im);
  }
  const cplx<R> x = valid ? cmake<R>((R)re, (R)im) : cmake<R>(R(0), R(0));
  // c' = V^H w' and ||w'||^2 (the first chunk from registers)
  double* P = D.part + (int64_t)s * str;
  chunk_dots<R, kVC>(v, x, valid, 0, j, wr, P + 2 * (m + 1), P + 4 * (m + 1) + 1, red);
  for (int kc = kVC; kc <= j; kc += kVC) {
    load_chunk<R, kVC>(V, M, ic, kc, j, v);
    chunk_dots<R, kVC>(v, x, valid, kc, j, wr, P + 2 * (m + 1), nullptr, red);
  }
  if (!wr) return;
  if (valid) as_global((cplx<R>*)D.basis)[(int64_t)(j + 1) * M + i] = x;
  if (ctr && threadIdx.x == 0) {
    const unsigned long long rows = min(kArnRows, M - s * kArnRows);
    atomicAdd(ctr, rows * (j + 3) * sizeof(cplx<R>));
  }
}

// The Hessenberg column of step j (one extra workgroup per system, running
// beside the row slices): h = c + c', h_{j+1} = ||w''||, previous rotations,
// new rotation, residual estimate.
__device__ __forceinline__ void arn_hessenberg(const SysDesc& D, int j, int S, int str) {
  __shared__ double c1[2 * (kMaxM + 1)], c2[2 * (kMaxM + 1)];
  __shared__ cf64 h[kMaxM + 2];
  __shared__ double rc_s[kMaxM];
  __shared__ cf64 rs_s[kMaxM];
  __shared__ double nsh[3];
  const int m = D.m, tid = threadIdx.x, lane = tid & 63;
  const CQM_GLOBAL double* part = as_global((const double*)D.part);
  const int n2j = 2 * (j + 1), T = 2 * n2j + 2;
  // task t: c (t < n2j), c' (t < 2 n2j), ||w||^2 and ||w'||^2
  auto task_off = [&](int t) -> int64_t {
    return t < n2j ? t : t < 2 * n2j ? 2 * (m + 1) + (t - n2j) : 4 * (m + 1) + (t - 2 * n2j);
  };
  auto task_put = [&](int t, double val) {
    if (t < n2j) c1[t] = val;
    else if (t < 2 * n2j) c2[t - n2j] = val;
    else nsh[t - 2 * n2j] = val;
  };
  const double val = slot_sum_g(part + task_off(min(tid, T - 1)), S, str);
  const int kq = min(tid, m - 1);
  const double rcv = as_global((const double*)D.cs)[kq];
  const cf64 rsv = as_global((const cf64*)D.sn)[kq];
  const cf64 gj = as_global((const cf64*)D.g)[j];
  const bool open = *as_global(D.sysi + 1) != 0;
  if (tid < T) task_put(tid, val);
  for (int t = tid + kArnRows; t < T; t += kArnRows) task_put(t, slot_sum_g(part + task_off(t), S, str));
  if (tid < j) {
    rc_s[tid] = rcv;
    rs_s[tid] = rsv;
  }
  __syncthreads();
  const bool second = nsh[1] < 0.49 * nsh[0];
  if (tid <= j)
    h[tid] = second ? cf64{c1[2 * tid] + c2[2 * tid], c1[2 * tid + 1] + c2[2 * tid + 1]}
                    : cf64{c1[2 * tid], c1[2 * tid + 1]};
  if (tid < 64) {
    double q = 0.0;
    if (second && lane <= j) q = c2[2 * lane] * c2[2 * lane] + c2[2 * lane + 1] * c2[2 * lane + 1];
    q = wave_sum(q);
    if (lane == 0) nsh[2] = second ? fmax(nsh[1] - q, 0.0) : nsh[1];
  }
  __syncthreads();
  if (!open || tid != 0) return;
  const double nr = sqrt(nsh[2]);
  h[j + 1] = cf64{nr, 0.0};
  hessenberg_column(D, j, h, rc_s, rs_s, gj, nr);
}

// Grid (S_max + 1, systems): x-blocks below S are row slices, the last one
// forms the Hessenberg column.  pre != 0 (FP32 inner steps): block-Jacobi
// preconditioned systems also form P v_{j+1} for the next step's product,
// into slot j + 2 (or zb), each wave for its own kSymB-row block (the block's
// inverse is loaded first, beside the slot sums).
static_assert(kArnRows == 4 * kSymB, "one diagonal block per wave of a row slice");
template <typename R, int kVC>
__global__ __launch_bounds__(kArnRows) void k_arn_finish(const SysDesc* __restrict__ sd, int j,
                                                        int pre, unsigned long long* ctr,
                                                        int* prog) {
  __shared__ double c2[2 * (kMaxM + 1)];
  __shared__ double nsh[3];
  __shared__ cplx<R> vz[kArnRows];
  step_progress(prog, j);
  const SysDesc D = sd[blockIdx.y];
  const int M = D.M, m = D.m;
  const int s = blockIdx.x;
  const int S = (M + kArnRows - 1) / kArnRows;
  const int str = arn_stride(m);
  if (s == (int)gridDim.x - 1) {
    arn_hessenberg(D, j, S, str);
    return;
  }
  const int tid = threadIdx.x, lane = tid & 63;
  const int i = s * kArnRows + tid;
  const bool valid = i < M;
  const int ic = valid ? i : M - 1;
  constexpr bool kCanFuse = sizeof(R) == 4;  // register budget
  const bool fuse = kCanFuse && pre && D.Pinv && j + 2 <= m;
  const int bw = s * (kArnRows / kSymB) + (tid >> 6);  // this wave's diagonal block
  const bool bin = bw * kSymB < M;
  cplx<R> pp[kCanFuse ? kSymB : 1];
  if constexpr (kCanFuse) {
    if (fuse && bin) pblock_load<R>((const cplx<R>*)D.Pinv + (int64_t)bw * kSymB * kSymB, lane, pp);
  }
  gcplx<R>* V = as_global((const cplx<R>*)D.basis);
  const cplx<R> x0 = V[(int64_t)(j + 1) * M + ic];
  // the first chunk is loaded before the second pass is known to be needed
  cplx<R> v[kVC];
  load_chunk<R, kVC>(V, M, ic, 0, j, v);
  // slot sums, task t: c' (t < 2 (j+1)), then ||w||^2 and ||w'||^2
  const CQM_GLOBAL double* part = as_global((const double*)D.part);
  const int n2j = 2 * (j + 1), T = n2j + 2;
  const double val = slot_sum_g(part + (min(tid, T - 1) < n2j ? 2 * (m + 1) + min(tid, T - 1)
                                                                 : 4 * (m + 1) + (min(tid, T - 1) - n2j)),
                                S, str);
  const bool wr = *as_global(D.sysi + 1) != 0 && s * kArnRows < M;
  if (tid < n2j) c2[tid] = val;
  else if (tid < T) nsh[tid - n2j] = val;
  for (int t = tid + kArnRows; t < n2j; t += kArnRows) c2[t] = slot_sum_g(part + 2 * (m + 1) + t, S, str);
  __syncthreads();
  const bool second = nsh[1] < 0.49 * nsh[0];
  if (tid < 64) {
    // ||w''||^2 = ||w'||^2 - ||c'||^2 (basis orthonormal); j + 1 <= 64 lanes
    double q = 0.0;
    if (second && lane <= j) q = c2[2 * lane] * c2[2 * lane] + c2[2 * lane + 1] * c2[2 * lane + 1];
    q = wave_sum(q);
    if (lane == 0) nsh[2] = second ? fmax(nsh[1] - q, 0.0) : nsh[1];
  }
  __syncthreads();
  const double nr = sqrt(nsh[2]);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  double re = x0.re, im = x0.im;
  if (second) {
    chunk_update<R, kVC>(v, 0, j, c2, re, im);
    for (int kc = kVC; kc <= j; kc += kVC) {
      load_chunk<R, kVC>(V, M, ic, kc, j, v);
      chunk_update<R, kVC>(v, kc, j, c2, re, im);
    }
  }
  if (!wr) return;
  const cplx<R> nv = cmake<R>((R)(re * inv), (R)(im * inv));
  if (valid) as_global((cplx<R>*)D.basis)[(int64_t)(j + 1) * M + i] = nv;
  if constexpr (kCanFuse) {
    if (fuse) {
      vz[tid] = valid ? nv : cmake<R>(R(0), R(0));
      __syncthreads();
      R zr = R(0), zi = R(0);
      if (bin) pblock_acc<R, R>(pp, vz + (tid & ~63), zr, zi);
      cplx<R>* z = D.zb ? (cplx<R>*)D.zb : (cplx<R>*)D.basis + (int64_t)(j + 2) * M;
      if (valid) as_global(z)[i] = cmake<R>(zr, zi);
    }
  }
  if (ctr && tid == 0) {
    const unsigned long long rows = min(kArnRows, M - s * kArnRows);
    // second pass and normalisation; with the next step's preconditioner
    // applied here, the rows of the diagonal-block inverse and the write
    atomicAdd(ctr, rows * ((second ? j + 3 : 2) + (fuse ? kSymB + 1 : 0)) * sizeof(cplx<R>));
  }
}

// Solution update of a finished cycle: y = R^-1 g (R the rotated Hessenberg
// factor, k x k upper triangular), then x += V_k y.  Grid (row slices of 256,
// systems); each slice's first wave solves the small triangular system
// (column-oriented: lane t holds the right-hand side entry t, y_i is
// broadcast and the lanes above subtract its column), then every thread
// updates one row of x.
template <typename R>
__global__ __launch_bounds__(256) void k_cycle_finish(const SysDesc* __restrict__ sd) {
  __shared__ cf64 y[kMaxM];
  __shared__ cf64 Hs[kMaxM * (kMaxM + 1) / 2];  // upper triangle, column by column
  const SysDesc D = sd[blockIdx.y];
  const int* st = D.sysi;
  if (!st[0]) return;
  const int k = st[2];
  if (k == 0) return;
  const int M = D.M, m = D.m;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= M) return;
  const cf64* Hl = D.H;
  // column t of the triangular factor holds rows 0..t: offset t (t+1) / 2
  for (int e = threadIdx.x; e < k * (k + 1) / 2; e += 256) {
    int t = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (t * (t + 1) / 2 > e) --t;
    while ((t + 1) * (t + 2) / 2 <= e) ++t;
    const int r = e - t * (t + 1) / 2;
    Hs[e] = Hl[(int64_t)(m + 1) * t + r];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int t = threadIdx.x;
    cf64 rhs = t < k ? D.g[t] : cf64{0.0, 0.0};
    // 1 / R_tt, one per lane
    cf64 inv{0.0, 0.0};
    if (t < k) {
      const cf64 d = Hs[t * (t + 1) / 2 + t];
      const double dn = d.re * d.re + d.im * d.im;
      inv = cf64{d.re / dn, -d.im / dn};
    }
    for (int c = k - 1; c >= 0; --c) {
      const cf64 a = t < c ? Hs[c * (c + 1) / 2 + t] : cf64{0.0, 0.0};
      const double yr0 = rhs.re * inv.re - rhs.im * inv.im;
      const double yi0 = rhs.re * inv.im + rhs.im * inv.re;
      const double yr = __shfl(yr0, c, 64), yi = __shfl(yi0, c, 64);
      if (t == c) y[c] = cf64{yr, yi};
      if (t < c) {
        rhs.re -= a.re * yr - a.im * yi;
        rhs.im -= a.re * yi + a.im * yr;
      }
    }
  }
  __syncthreads();
  const cplx<R>* V = (const cplx<R>*)D.basis;
  const bool valid = i < M;
  double re = 0.0, im = 0.0;
  basis_combine<R, 16>(V, M, valid ? i : M - 1, y, k, 1.0, re, im);  // (V y)_i
  if (!D.Pinv) {
    if (valid) {
      const cf64 xv = D.x[i];
      D.x[i] = cf64{xv.re + re, xv.im + im};
    }
    return;
  }
  // right preconditioning: x += P (V y); a workgroup's 256 rows are four
  // whole diagonal blocks, one per wave
  __shared__ cf64 vy[256];
  vy[threadIdx.x] = valid ? cf64{re, im} : cf64{0.0, 0.0};
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + w;
  if (b * kSymB >= M) return;
  double zr = 0.0, zi = 0.0;
  pblock_mul<R, double, 16>((const cplx<R>*)D.Pinv + (int64_t)b * kSymB * kSymB, vy + w * kSymB,
                            lane, zr, zi);
  if (valid) {
    const cf64 xv = D.x[i];
    D.x[i] = cf64{xv.re + zr, xv.im + zi};
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
void launch_gather_diag(const SysDesc* sd, int n, int* flags, double* norms, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_diag, dim3((n + 255) / 256), dim3(256), 0, s, sd, n, flags, norms);
  CQM_HIP(hipGetLastError());
}
template <typename R>
void launch_cycle_start(const SysDesc* sd, int n, double outer_tol, double inner_tol, double relax,
                        hipStream_t s) {
  hipLaunchKernelGGL((k_cycle_start<R>), dim3(n), dim3(256), 0, s, sd, outer_tol, inner_tol, relax);
  CQM_HIP(hipGetLastError());
}
// One workgroup per system, or the three launches over row slices (the
// finish launch has one more x-block per system for the Hessenberg column).
template <typename R>
void launch_arnoldi(const SysDesc* sd, int n, int maxM, int j, bool split, bool fused,
                    bool pre, unsigned long long* ctr, int* prog, hipStream_t s) {
  const int pf = pre ? 1 : 0;
  const int f = fused ? 1 : 0;
  if (split) {
    const int S = (maxM + kArnRows - 1) / kArnRows;
    const dim3 grid(S, n), gfin(S + 1, n), blk(kArnRows);
    if (j < 16) {
      hipLaunchKernelGGL((k_arn_dots<R, 16>), grid, blk, 0, s, sd, j, f, ctr);
      hipLaunchKernelGGL((k_arn_update<R, 16>), grid, blk, 0, s, sd, j, ctr);
      hipLaunchKernelGGL((k_arn_finish<R, 16>), gfin, blk, 0, s, sd, j, pf, ctr, prog);
    } else {
      hipLaunchKernelGGL((k_arn_dots<R, 32>), grid, blk, 0, s, sd, j, f, ctr);
      hipLaunchKernelGGL((k_arn_update<R, 32>), grid, blk, 0, s, sd, j, ctr);
      hipLaunchKernelGGL((k_arn_finish<R, 32>), gfin, blk, 0, s, sd, j, pf, ctr, prog);
    }
  } else if (maxM < 3072) {
    hipLaunchKernelGGL((k_arnoldi<R, 256>), dim3(n), dim3(256), 0, s, sd, j, ctr, prog);
  } else {
    hipLaunchKernelGGL((k_arnoldi<R, 1024>), dim3(n), dim3(1024), 0, s, sd, j, ctr, prog);
  }
  CQM_HIP(hipGetLastError());
}
template <typename R> void launch_cycle_finish(const SysDesc* sd, int n, int maxM, hipStream_t s) {
  hipLaunchKernelGGL((k_cycle_finish<R>), dim3((maxM + 255) / 256, n), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}

template void launch_cycle_start<float>(const SysDesc*, int, double, double, double, hipStream_t);
template void launch_cycle_start<double>(const SysDesc*, int, double, double, double, hipStream_t);
template void launch_arnoldi<float>(const SysDesc*, int, int, int, bool, bool, bool,
                                    unsigned long long*, int*, hipStream_t);
template void launch_arnoldi<double>(const SysDesc*, int, int, int, bool, bool, bool,
                                     unsigned long long*, int*, hipStream_t);
template void launch_cycle_finish<float>(const SysDesc*, int, int, hipStream_t);
template void launch_cycle_finish<double>(const SysDesc*, int, int, hipStream_t);

}  // namespace cqm

