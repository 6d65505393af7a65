// Time-marching solve of the convolution system of Section 3.2 for the
// indirect single-layer form: the integration weights
//   What_n = rho^-n / F  sum_{l<F} V(s_l) zeta^(n l)        (eq. dft, F = N+1)
// from the stored operator, the history sums of eq. cqmrhs
//   r_n = b_n - sum_{j=1}^{n} What_j q_{n-j},
// and What_0 q_n = r_n (real symmetric positive definite) by preconditioned
// conjugate gradients with the inverses of What_0's 64 x 64 diagonal blocks.
//
// The weights are real and keep the stored operator's layout: the upper
// triangle of 64 x 64 tiles, tile (I, J) at J (J+1)/2 + I, row-major inside,
// one slice of sym_slice(M) doubles per n.  Products with them use the
// tile-partial scheme of the complex products: one workgroup per tile (and
// per chunk of weights), row sums into P[.][J][rows of I], column sums into
// P[.][I][rows of J], summed per row in a fixed order afterwards.
#include "device_util.h"

namespace cqm {

namespace {
constexpr int kB = kSymB;
constexpr int kRows = kB / 4;  // rows per wave of a tile
constexpr int kWE = 16;        // entries per workgroup of the weight transform
constexpr int kWL = 64;        // frequencies staged in LDS per round

__device__ __forceinline__ void decode_tile_m(int t, int& I, int& J) {
  int jj = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
  while (jj * (jj + 1) / 2 > t) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= t) ++jj;
  J = jj;
  I = t - jj * (jj + 1) / 2;
}
}  // namespace

// What_n[e] = (rho^-n / F) Re( sum_{l<F} V_l[e] zeta^(n l) ) with the
// conjugate frequencies folded in (V_{F-l} = conj V_l):
//   = (rho^-n / F) [ Re V_0[e] + sum_{l=1}^{H-1} c_l Re(V_l[e] zeta^(n l)) ],
// c_l = 2, or 1 for l = F/2 when F is even.  Thread (entry ie, lane in)
// forms n = nbase + in + 16 k, k < NW; the stored frequencies of 16 entries
// are staged through LDS 64 at a time.
template <int NW>
__global__ __launch_bounds__(256) void k_march_weights(const cf64* __restrict__ V, int64_t SL, int H,
                                                       int F, const cf64* __restrict__ tw,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ W) {
  __shared__ cf64 vs[kWE][kWL + 1];  // padded row: no bank conflicts between entries
  const int ie = threadIdx.x % kWE, in = threadIdx.x / kWE;
  const int64_t e0 = (int64_t)blockIdx.x * kWE;
  const int nbase = blockIdx.y * (16 * NW);
  int idx[NW], inc[NW];
  double acc[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int n = nbase + in + 16 * k;
    inc[k] = n < F ? n : 0;  // (n l) mod F advances by n per frequency
    idx[k] = 0;
    acc[k] = 0.0;
  }
  for (int l0 = 0; l0 < H; l0 += kWL) {
    const int nl = min(kWL, H - l0);
    __syncthreads();
    for (int k = threadIdx.x; k < kWE * nl; k += 256) {
      const int li = k / kWE, ei = k % kWE;  // consecutive threads: consecutive entries
      const int64_t e = e0 + ei;
      vs[ei][li] = e < SL ? V[(int64_t)(l0 + li) * SL + e] : cf64{0.0, 0.0};
    }
    __syncthreads();
    for (int li = 0; li < nl; ++li) {
      const int l = l0 + li;
      const cf64 v = vs[ie][li];
      const double c = (l == 0 || 2 * l == F) ? 1.0 : 2.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const cf64 z = tw[idx[k]];
        acc[k] = fma(c, v.re * z.re - v.im * z.im, acc[k]);
        idx[k] += inc[k];
        if (idx[k] >= F) idx[k] -= F;
      }
    }
  }
  const int64_t e = e0 + ie;
  if (e >= SL) return;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int n = nbase + in + 16 * k;
    if (n < F) W[(int64_t)n * SL + e] = acc[k] * scale[n];
  }
}

// Tile partial sums of  sum_{j < cnt} W_{j0 + j} x_{xb - j}  (x rows of
// length M in X), weights j of chunk s = blockIdx.y: j in [s jc, s jc + jc).
// P[s][Y][nb kB] receives every slot once.  Entries outside [0, M)^2 are
// masked (the tile padding is not data).  A set *done flag skips the launch
// (conjugate gradients after convergence).
__global__ __launch_bounds__(256) void k_march_gemv(const double* __restrict__ W, int64_t SL, int M,
                                                    int j0, int cnt, int jc,
                                                    const double* __restrict__ X, int xb,
                                                    double* __restrict__ P,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double colred[4][kB];
  const int t = blockIdx.x, s = blockIdx.y;
  int I, J;
  decode_tile_m(t, I, J);
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nb = sym_blocks(M);
  const int jb = s * jc, je = min(cnt, jb + jc);
  const bool col_in = J * kB + c < M;
  double racc[kRows];
#pragma unroll
  for (int q = 0; q < kRows; ++q) racc[q] = 0.0;
  double cacc = 0.0;
  for (int j = jb; j < je; ++j) {
    const double* T = W + (int64_t)(j0 + j) * SL + (int64_t)t * kB * kB;
    const double* x = X + (int64_t)(xb - j) * M;
    const double xj = col_in ? x[J * kB + c] : 0.0;
    const double xi = I * kB + c < M ? x[I * kB + c] : 0.0;
    double a[kRows];
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int r = w * kRows + q;
      const double v = as_global(T)[r * kB + c];
      a[q] = (I * kB + r < M && col_in) ? v : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      racc[q] = fma(a[q], xj, racc[q]);
      cacc = fma(a[q], lane_bcast(xi, w * kRows + q), cacc);
    }
  }
  const int64_t ntB = (int64_t)nb * kB;
  double* Ps = P + (int64_t)s * nb * ntB;
  // rows of I: the wave's 16 row sums over its 64 lanes
  wave_reduce_scatter_near<kRows>(racc, c);
  if (c < kRows) Ps[(int64_t)J * ntB + I * kB + w * kRows + scatter_entry<kRows>(c)] = racc[0];
  if (I != J) {
    colred[w][c] = cacc;
    __syncthreads();
    if (w == 0)
      Ps[(int64_t)I * ntB + J * kB + c] = (colred[0][c] + colred[1][c]) + (colred[2][c] + colred[3][c]);
  }
}

// y_i = add_i + sign * sum_{s < S} sum_{Y < nb} P[s][Y][i]  (fixed order).
__global__ __launch_bounds__(256) void k_march_reduce(const double* __restrict__ P, int S, int M,
                                                      double sign, const double* __restrict__ add,
                                                      double* __restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int nb = sym_blocks(M);
  const int64_t ntB = (int64_t)nb * kB;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += slot_sum(P + (int64_t)s * nb * ntB + i, nb, ntB);
  y[i] = (add ? add[i] : 0.0) + sign * acc;
}

// The diagonal tiles of What_0 as complex blocks [block][kB][kB] (imaginary
// part zero) for the block inverse of the stored form.
__global__ __launch_bounds__(256) void k_march_diag(const double* __restrict__ W0, int M,
                                                    cf64* __restrict__ out) {
  const int b = blockIdx.x;
  const double* T = W0 + (int64_t)(b * (b + 1) / 2 + b) * kB * kB;
  for (int k = threadIdx.x; k < kB * kB; k += 256)
    out[(int64_t)b * kB * kB + k] = cf64{T[k], 0.0};
}

// ------------------------------------------------------------------ PCG
// Conjugate gradients for What_0 q = r (CgVec, internal.h): x (the step's
// row of q), r, z = P r, p, w = What_0 p; per-workgroup partial sums
// (workgroups of 256 rows = 4 diagonal blocks, so z of a workgroup's rows
// needs only its own r): rz[2][nwg] (by iteration parity), pw[nwg], rr[nwg],
// bb[nwg].  Scalars are re-formed by every workgroup from the partials in a
// fixed order.

namespace {
__device__ __forceinline__ double psum(const double* a, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += a[k];
  return s;
}
// z of the workgroup's rows: z_r = sum_c Pinv[c][r] r_c per diagonal block
// (one block per wave; Pinv symmetric up to rounding, one orientation)
__device__ __forceinline__ void block_apply_rows(const CgVec& v, int row0, double* rs) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = row0 / kB + w;
  const int i = row0 + threadIdx.x;
  rs[threadIdx.x] = i < v.M ? v.r[i] : 0.0;
  __syncthreads();
  if (b * kB < v.M) {
    const cf64* Pb = v.pinv + (int64_t)b * kB * kB;
    double acc = 0.0;
    for (int c = 0; c < kB; ++c) acc = fma(Pb[c * kB + lane].re, rs[w * kB + c], acc);
    if (i < v.M) v.z[i] = acc;
  }
  __syncthreads();
}
}  // namespace

// Start: x = 0, z = P r, p = z; partials rz[0], rr, bb = r.r; flags cleared.
__global__ __launch_bounds__(256) void k_cg_init(CgVec v) {
  __shared__ double rs[256];
  __shared__ double red[16];
  const int row0 = blockIdx.x * 256, i = row0 + threadIdx.x;
  if (i < v.M) v.x[i] = 0.0;
  block_apply_rows(v, row0, rs);
  const double ri = i < v.M ? v.r[i] : 0.0, zi = i < v.M ? v.z[i] : 0.0;
  if (i < v.M) v.p[i] = zi;
  const double rz = block_sum(ri * zi, red);
  const double rr = block_sum(ri * ri, red);
  if (threadIdx.x == 0) {
    v.rz[blockIdx.x] = rz;
    v.rr[blockIdx.x] = rr;
    v.bb[blockIdx.x] = rr;
    if (blockIdx.x == 0) {
      *v.done = 0;
      *v.iters = 0;
    }
  }
}

// Convergence test at the start of an iteration (every workgroup of the
// product forms it identically): ||r||^2 <= tol^2 ||r_0||^2 sets the flags.
__device__ __forceinline__ bool cg_converged(const CgVec& v, double tol2) {
  const double rr = psum(v.rr, v.nwg), bb = psum(v.bb, v.nwg);
  return !(rr > tol2 * bb) || !isfinite(rr);
}

__global__ void k_cg_check(CgVec v, double tol2) {
  if (*v.done) return;
  if (cg_converged(v, tol2)) {
    *v.done = 1;
    __threadfence_system();
    *(volatile int*)v.hdone = 1;
  }
}

// w = What_0 p (rows of this workgroup) from the product's partials, and the
// partial p.w.
__global__ __launch_bounds__(256) void k_cg_reduce(CgVec v, const double* __restrict__ P) {
  if (*v.done) return;
  __shared__ double red[16];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int nb = sym_blocks(v.M);
  const int64_t ntB = (int64_t)nb * kB;
  double wi = 0.0, pi = 0.0;
  if (i < v.M) {
    wi = slot_sum(P + i, nb, ntB);
    pi = v.p[i];
    v.w[i] = wi;
  }
  const double pw = block_sum(pi * wi, red);
  if (threadIdx.x == 0) v.pw[blockIdx.x] = pw;
}

// alpha = rz / pw; x += alpha p, r -= alpha w; z = P r; partial r.z into
// rz[par ^ 1] and r.r; then beta = rz_new / rz_old and p = z + beta p for the
// workgroup's rows (the next product reads p only after this launch).
__global__ __launch_bounds__(256) void k_cg_update(CgVec v, int par) {
  if (*v.done) return;
  __shared__ double rs[256];
  __shared__ double red[16];
  const int row0 = blockIdx.x * 256, i = row0 + threadIdx.x;
  const double alpha = psum(v.rz + par * v.nwg, v.nwg) / psum(v.pw, v.nwg);
  if (i < v.M) {
    v.x[i] = fma(alpha, v.p[i], v.x[i]);
    v.r[i] = fma(-alpha, v.w[i], v.r[i]);
  }
  __syncthreads();
  block_apply_rows(v, row0, rs);
  const double ri = i < v.M ? v.r[i] : 0.0, zi = i < v.M ? v.z[i] : 0.0;
  const double rz = block_sum(ri * zi, red);
  const double rr = block_sum(ri * ri, red);
  if (threadIdx.x == 0) {
    v.rz[(par ^ 1) * v.nwg + blockIdx.x] = rz;
    v.rr[blockIdx.x] = rr;
    if (blockIdx.x == 0) *v.iters += 1;
  }
}

// p = z + beta p with beta = rz_new / rz_old (all partials of the update are
// in place once this launch starts).
__global__ __launch_bounds__(256) void k_cg_direction(CgVec v, int par) {
  if (*v.done) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double beta = psum(v.rz + (par ^ 1) * v.nwg, v.nwg) / psum(v.rz + par * v.nwg, v.nwg);
  if (i < v.M) v.p[i] = fma(beta, v.p[i], v.z[i]);
}

// ------------------------------------------------------------------ compressed marching
// r = b - sum_{k < n} Re Y[k] (the history sum of eq. cqmrhs from the
// compressed weights' products, one row per lag)
__global__ __launch_bounds__(256) void k_hist_reduce(const cf64* __restrict__ Y, int n, int M,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  double acc = 0.0;
  for (int k = 0; k < n; ++k) acc += Y[(int64_t)k * M + i].re;
  r[i] = b[i] - acc;
}

// z = x + 0 i (skipped once the CG has converged)
__global__ __launch_bounds__(256) void k_to_complex(const double* __restrict__ x, int M,
                                                    cf64* __restrict__ z, const int* done) {
  if (done && *done) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < M) z[i] = cf64{x[i], 0.0};
}

// w = Re y (the real weight's product with the real direction) and the
// partial p.w of the workgroup's rows
__global__ __launch_bounds__(256) void k_cg_reduce_complex(CgVec v, const cf64* __restrict__ y) {
  if (*v.done) return;
  __shared__ double red[16];
  const int i = blockIdx.x * 256 + threadIdx.x;
  double wi = 0.0, pi = 0.0;
  if (i < v.M) {
    wi = y[i].re;
    pi = v.p[i];
    v.w[i] = wi;
  }
  const double pw = block_sum(pi * wi, red);
  if (threadIdx.x == 0) v.pw[blockIdx.x] = pw;
}

// out = Re (1/F) sum_l blocks[l] (the plain operator's diagonal blocks at
// every frequency: their mean is the diagonal block of What_0, eq. dft at
// n = 0)
__global__ __launch_bounds__(256) void k_freq_mean_blocks(const cf64* __restrict__ blocks, int F,
                                                          int64_t nel, cf64* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nel) return;
  double acc = 0.0;
  for (int l = 0; l < F; ++l) acc += blocks[(int64_t)l * nel + e].re;
  out[e] = cf64{acc / F, 0.0};
}

void launch_hist_reduce(const cf64* Y, int n, int M, const double* b, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_hist_reduce, dim3((M + 255) / 256), dim3(256), 0, s, Y, n, M, b, r);
  CQM_HIP(hipGetLastError());
}
void launch_to_complex(const double* x, int M, cf64* z, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_to_complex, dim3((M + 255) / 256), dim3(256), 0, s, x, M, z, done);
  CQM_HIP(hipGetLastError());
}
void launch_cg_reduce_complex(const CgVec& v, const cf64* y, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_reduce_complex, dim3(v.nwg), dim3(256), 0, s, v, y);
  CQM_HIP(hipGetLastError());
}
void launch_freq_mean_blocks(const cf64* blocks, int F, int64_t nel, cf64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_freq_mean_blocks, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s, blocks,
                     F, nel, out);
  CQM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ launchers
void launch_march_weights(const cf64* V, int M, int H, int F, const cf64* tw, const double* scale,
                          double* W, hipStream_t s) {
  const int64_t SL = sym_slice(M);
  const unsigned gx = (unsigned)((SL + kWE - 1) / kWE);
  if (F <= 16 * 5) {
    hipLaunchKernelGGL(k_march_weights<5>, dim3(gx, 1), dim3(256), 0, s, V, SL, H, F, tw, scale, W);
  } else {
    const unsigned gy = (unsigned)((F + 16 * 9 - 1) / (16 * 9));
    hipLaunchKernelGGL(k_march_weights<9>, dim3(gx, gy), dim3(256), 0, s, V, SL, H, F, tw, scale, W);
  }
  CQM_HIP(hipGetLastError());
}

int march_chunks(int M, int cnt) {
  // enough workgroups to fill the chip: tiles x chunks >= 2048
  const int tiles = sym_tiles(M);
  int S = (2048 + tiles - 1) / tiles;
  S = std::max(1, std::min(S, cnt));
  return S;
}

void launch_march_product(const double* W, int M, int j0, int cnt, const double* X, int xb,
                          double* P, int S, const int* done, hipStream_t s) {
  const int jc = (cnt + S - 1) / S;
  hipLaunchKernelGGL(k_march_gemv, dim3(sym_tiles(M), S), dim3(256), 0, s, W, sym_slice(M), M, j0,
                     cnt, jc, X, xb, P, done);
  CQM_HIP(hipGetLastError());
}

void launch_march_reduce(const double* P, int S, int M, double sign, const double* add, double* y,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_march_reduce, dim3((M + 255) / 256), dim3(256), 0, s, P, S, M, sign, add, y);
  CQM_HIP(hipGetLastError());
}

void launch_march_diag(const double* W0, int M, cf64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_march_diag, dim3(sym_blocks(M)), dim3(256), 0, s, W0, M, out);
  CQM_HIP(hipGetLastError());
}

void launch_cg_init(const CgVec& v, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(v.nwg), dim3(256), 0, s, v);
  CQM_HIP(hipGetLastError());
}

// One iteration: convergence test, product What_0 p, w and p.w, update of x,
// r and z, new direction.  Every launch leaves at once after convergence.
void launch_cg_iteration(const CgVec& v, const double* W0, double* P, int par, double tol2,
                         hipStream_t s) {
  const int M = v.M;
  hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(1), 0, s, v, tol2);
  hipLaunchKernelGGL(k_march_gemv, dim3(sym_tiles(M), 1), dim3(256), 0, s, W0, sym_slice(M), M, 0, 1,
                     1, (const double*)v.p, 0, P, (const int*)v.done);
  hipLaunchKernelGGL(k_cg_reduce, dim3(v.nwg), dim3(256), 0, s, v, (const double*)P);
  hipLaunchKernelGGL(k_cg_update, dim3(v.nwg), dim3(256), 0, s, v, par);
  hipLaunchKernelGGL(k_cg_direction, dim3(v.nwg), dim3(256), 0, s, v, par);
  CQM_HIP(hipGetLastError());
}

// The CG iteration's parts around an external product (the compressed
// marching): the convergence test, then, after w = What_0 p, the update and
// the new direction.
void launch_cg_check(const CgVec& v, double tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(1), 0, s, v, tol2);
  CQM_HIP(hipGetLastError());
}
void launch_cg_finish(const CgVec& v, int par, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update, dim3(v.nwg), dim3(256), 0, s, v, par);
  hipLaunchKernelGGL(k_cg_direction, dim3(v.nwg), dim3(256), 0, s, v, par);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
