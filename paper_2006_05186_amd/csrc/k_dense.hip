// Stored dense operator.  The Galerkin single-layer matrix V(s) is complex
// symmetric (the kernel depends on |x - y| only and trial and test spaces
// coincide, Section 2), so only its upper triangle of kSymB x kSymB tiles is
// kept: tile (I, J), I <= J, at index J (J + 1) / 2 + I, row-major inside, so
// the tiles of block column J are contiguous.
//
// y = V x tile by tile: one workgroup reads tile (I, J) once and forms
//   rows of block I:  V_IJ x_J        -> P[J][rows of I]
//   rows of block J:  V_IJ^T x_I      -> P[I][rows of J]   (I < J)
// so every slot of the partial buffer P (nt slots of nt kSymB rows) is
// written exactly once, and a second kernel sums y_i = sum_Y P[Y][i] in a
// fixed order: no atomics, deterministic, half the operator bytes of a full
// row-major product.  Entries outside [0, M)^2 (ragged last block) are masked,
// so tile padding is never read as data.
#include <algorithm>

#include "device_util.h"

namespace cqm {

namespace {
constexpr int kB = kSymB;
constexpr int kRowsPerWave = kB / 4;  // 4 waves per tile, 16 rows each

// The tile's values held by this thread: 16 rows per wave, one column per
// lane (each row read by a wave is 64 contiguous entries).
template <typename R>
__device__ __forceinline__ void load_tile(const cplx<R>* __restrict__ Vt, cplx<R>* a) {
  // each operator entry is read once per product: non-temporal loads keep
  // the stream from evicting the vectors and partial sums
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  typedef R v2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(Vt) + (w * kRowsPerWave + q) * kB + c);
    a[q].re = v.x;
    a[q].im = v.y;
  }
}

template <typename R>
__device__ __forceinline__ cplx<R> load_x(const cplx<R>* __restrict__ x, int g, int M) {
  cplx<R> v;
  v.re = R(0);
  v.im = R(0);
  if (g < M) v = as_global(x)[g];
  return v;
}

// Row sums of a masked tile with x_J (value xj of this lane's column): the
// wave's 16 rows reduced over its 64 lanes and stored to prow[0..15].
template <typename R>
__device__ __forceinline__ void tile_row_sums(const cplx<R>* a, cplx<R> xj, R* prow, int c) {
  if constexpr (sizeof(R) == 4) {
    R v[2 * kRowsPerWave];
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      v[q] = a[q].re * xj.re - a[q].im * xj.im;
      v[kRowsPerWave + q] = a[q].re * xj.im + a[q].im * xj.re;
    }
    wave_reduce_scatter_near<2 * kRowsPerWave>(v, c);
    if (c < 2 * kRowsPerWave) {
      const int e = scatter_entry<2 * kRowsPerWave>(c);
      prow[2 * (e % kRowsPerWave) + e / kRowsPerWave] = v[0];
    }
  } else {
    // FP64: real and imaginary parts in two rounds (register budget)
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      R v[kRowsPerWave];
#pragma unroll
      for (int q = 0; q < kRowsPerWave; ++q)
        v[q] = part == 0 ? a[q].re * xj.re - a[q].im * xj.im : a[q].re * xj.im + a[q].im * xj.re;
      wave_reduce_scatter_near<kRowsPerWave>(v, c);
      if (c < kRowsPerWave) prow[2 * scatter_entry<kRowsPerWave>(c) + part] = v[0];
    }
  }
}

__device__ __forceinline__ void decode_tile(int t, int& I, int& J) {
  int jj = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
  while (jj * (jj + 1) / 2 > t) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= t) ++jj;
  J = jj;
  I = t - jj * (jj + 1) / 2;
}

// Both contributions of one loaded tile (I, J) for one input vector x:
// row sums into P[J][rows of I], column sums (off-diagonal tiles) into
// P[I][rows of J].  x_I and x_J are read one entry per lane; the rows' x_I
// values are broadcast from their lanes.
template <typename R>
__device__ __forceinline__ void tile_products(const cplx<R>* a, int M, int I, int J,
                                              const cplx<R>* __restrict__ x, cplx<R>* P, int ntB,
                                              cplx<R> (*colred)[kB]) {
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const cplx<R> xj = load_x<R>(x, J * kB + c, M);
  tile_row_sums<R>(a, xj, reinterpret_cast<R*>(P + (int64_t)J * ntB + I * kB + w * kRowsPerWave),
                   c);
  if (I != J) {
    const cplx<R> xi = load_x<R>(x, I * kB + c, M);
    R cre = R(0), cim = R(0);
#pragma unroll
    for (int q = 0; q < kRowsPerWave; ++q) {
      const int r = w * kRowsPerWave + q;
      const R xr = lane_bcast(xi.re, r), xm = lane_bcast(xi.im, r);  // r is wave-uniform
      cre += a[q].re * xr - a[q].im * xm;
      cim += a[q].re * xm + a[q].im * xr;
    }
    colred[w][c].re = cre;
    colred[w][c].im = cim;
    __syncthreads();
    if (w == 0) {
      cplx<R> o;
      o.re = (colred[0][c].re + colred[1][c].re) + (colred[2][c].re + colred[3][c].re);
      o.im = (colred[0][c].im + colred[1][c].im) + (colred[2][c].im + colred[3][c].im);
      P[(int64_t)I * ntB + J * kB + c] = o;
    }
    __syncthreads();
  }
}

// Load tile t of a slice and mask the entries outside [0, M)^2.
template <typename R>
__device__ __forceinline__ void masked_tile(const cplx<R>* __restrict__ Vs, int t, int M, int I,
                                            int J, cplx<R>* a) {
  load_tile<R>(Vs + (int64_t)t * kB * kB, a);
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const bool col_in = J * kB + c < M;
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    const bool in = (I * kB + w * kRowsPerWave + q < M) && col_in;
    a[q].re = in ? a[q].re : R(0);
    a[q].im = in ? a[q].im : R(0);
  }
}

template <typename R>
__device__ __forceinline__ cplx<R> sum_partials(const cplx<R>* __restrict__ P, int M, int i) {
  return sym_row_sum<R>(P, M, i);
}
}  // namespace

// ------------------------------------------------------------ plain form
// y_l = V_l x_l for frequencies l < nsys (slices V + l * sym_slice(M)).
template <typename R>
__global__ __launch_bounds__(256) void k_symv(const cplx<R>* __restrict__ V, int M,
                                              const cplx<R>* __restrict__ x, int64_t xs,
                                              cplx<R>* __restrict__ part,
                                              const int* __restrict__ active) {
  __shared__ cplx<R> colred[4][kB];
  const int l = blockIdx.y;
  if (active && !active[l * kSysiStride]) return;
  const int t = blockIdx.x;
  int I, J;
  decode_tile(t, I, J);
  cplx<R> a[kRowsPerWave];
  masked_tile<R>(V + (int64_t)l * sym_slice(M), t, M, I, J, a);
  tile_products<R>(a, M, I, J, x + (int64_t)l * xs, part + (int64_t)l * sym_partials(M),
                   sym_blocks(M) * kB, colred);
}

template <typename R>
__global__ __launch_bounds__(256) void k_symv_reduce(const cplx<R>* __restrict__ part, int M,
                                                     cplx<R>* __restrict__ y, int64_t ys,
                                                     const int* __restrict__ active) {
  const int l = blockIdx.y;
  if (active && !active[l * kSysiStride]) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  y[(int64_t)l * ys + i] = sum_partials<R>(part + (int64_t)l * sym_partials(M), M, i);
}

template <typename R>
void launch_dense_gemv(const cplx<R>* V, int M, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y,
                       int64_t ys, const int* active, cplx<R>* part, hipStream_t s) {
  hipLaunchKernelGGL((k_symv<R>), dim3(sym_tiles(M), nsys), dim3(256), 0, s, V, M, x, xs, part,
                     active);
  hipLaunchKernelGGL((k_symv_reduce<R>), dim3((M + 255) / 256, nsys), dim3(256), 0, s, part, M, y,
                     ys, active);
  CQM_HIP(hipGetLastError());
}

// ------------------------------------------------------------ descriptors
// Products over system groups (a group: systems sharing one operator slice,
// up to kMaxGroup).  The host launches one grid per mesh size, (tiles x open
// groups), each workgroup reading its group record once: the tile, the
// members' flags and vectors all hang off that one load.  The group lists
// are rebuilt by the host at its status checks; members closed since are
// skipped.  which = 0: basis[j] -> basis[j+1] of systems with an open cycle
// (inner precision); which = 1: x -> r = ghat - V x of open systems whose
// residual is not formed in double-double this cycle (FP64).
__device__ __forceinline__ bool member_on(const int* sysi, int which) {
  return which == 0 ? sysi[1] != 0 : (sysi[0] != 0 && sysi[4] == 0);
}
template <typename R, bool kGrouped>
__global__ __launch_bounds__(256) void k_symv_groups(const GroupLite* __restrict__ gl, int which,
                                                     int j, unsigned long long* ctr) {
  __shared__ cplx<R> colred[4][kB];
  const GroupLite& G = gl[blockIdx.y];
  const int M = G.M;
  const int t = blockIdx.x;
  {
    // groups with no open member leave at once (the full list is used by
    // graph-captured steps)
    bool any = false;
    for (int k = 0; k < (kGrouped ? G.n : 1); ++k) any |= member_on(G.sysi[k], which);
    if (!any) return;
  }
  int I, J;
  decode_tile(t, I, J);
  const int ntB = sym_blocks(M) * kB;
  const int n = kGrouped ? G.n : 1;
  // cut-off: a tile whose blocks' box gap reaches the slice's radius holds
  // only zeros (the assembly left those entries out); its partial sums are
  // zero and it is not read
  if (G.gap && G.gap[t] >= (which == 0 && sizeof(R) == 4 ? G.cut32 : G.cut64)) {
    if (threadIdx.x < kB) {
      cplx<R> z;
      z.re = R(0);
      z.im = R(0);
      for (int k = 0; k < n; ++k) {
        if (!member_on(G.sysi[k], which)) continue;
        cplx<R>* P = (cplx<R>*)G.symp[k];
        P[(int64_t)J * ntB + I * kB + threadIdx.x] = z;
        if (I != J) P[(int64_t)I * ntB + J * kB + threadIdx.x] = z;
      }
    }
    return;
  }
  const void* Vs = which == 0 ? (sizeof(R) == 4 ? G.V32 : G.V64) : G.V64;
  cplx<R> a[kRowsPerWave];
  masked_tile<R>((const cplx<R>*)Vs, t, M, I, J, a);
  int done = 0;
  for (int k = 0; k < n; ++k) {
    if (!member_on(G.sysi[k], which)) continue;
    const cplx<R>* x = which == 0 ? (const cplx<R>*)G.basis[k] + (int64_t)j * M
                                  : (const cplx<R>*)(const void*)G.x[k];
    tile_products<R>(a, M, I, J, x, (cplx<R>*)G.symp[k], ntB, colred);
    ++done;
  }
  if (ctr && t == 0 && threadIdx.x == 0 && done) {
    // algorithmic bytes, charged once per group by its first tile (never
    // left out): the entries of the upper triangle a product reads under the
    // slice's cut-off (counted by the host), each member's vectors once
    const long long e = which == 0 && sizeof(R) == 4 ? G.entries32 : G.entries64;
    atomicAdd(ctr, ((unsigned long long)e + (unsigned long long)done * 2 * (unsigned long long)M) *
                       sizeof(cplx<R>));
  }
}

// FP64 refinement residual r = ghat - V x in double-double arithmetic:
// every product exact (two_prod), every sum carried to ~106 bits, the
// partial sums stored as (hi, lo) pairs (P_hi in the first sym_partials
// slots of the member's buffer, P_lo in the next), r rounded once.  With the
// residual formed in FP64 the refinement stalls where the rounding of V x
// (about 1e-16 of |V||x|) hides the true residual, and the time-domain
// solution, which amplifies per-frequency errors by up to rho^-N, inherits
// that floor; formed in double-double, x converges to the solution of the
// stored FP64 system.
// open systems whose closing residual is formed in double-double
__device__ __forceinline__ bool dd_on(const int* sysi) { return sysi[0] != 0 && sysi[4] != 0; }

__global__ __launch_bounds__(256) void k_symv_resid_dd(const GroupLite* __restrict__ gl, int grouped,
                                                       unsigned long long* ctr) {
  __shared__ dd colred[4][kB][2];
  const GroupLite& G = gl[blockIdx.y];
  const int M = G.M;
  const int t = blockIdx.x;
  const int n = grouped ? G.n : 1;
  {
    bool any = false;
    for (int k = 0; k < n; ++k) any |= dd_on(G.sysi[k]);
    if (!any) return;
  }
  int I, J;
  decode_tile(t, I, J);
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ntB = sym_blocks(M) * kB;
  const int64_t np = sym_partials(M);
  if (G.gap && G.gap[t] >= G.cut64) {
    // a tile left out by the cut-off holds only zeros
    if (threadIdx.x < kB) {
      for (int k = 0; k < n; ++k) {
        if (!dd_on(G.sysi[k])) continue;
        cf64* P = (cf64*)G.symp[k];
        P[(int64_t)J * ntB + I * kB + threadIdx.x] = cf64{0.0, 0.0};
        P[np + (int64_t)J * ntB + I * kB + threadIdx.x] = cf64{0.0, 0.0};
        if (I != J) {
          P[(int64_t)I * ntB + J * kB + threadIdx.x] = cf64{0.0, 0.0};
          P[np + (int64_t)I * ntB + J * kB + threadIdx.x] = cf64{0.0, 0.0};
        }
      }
    }
    return;
  }
  cf64 a[kRowsPerWave];
  masked_tile<double>((const cf64*)G.V64, t, M, I, J, a);
  if (ctr && t == 0 && threadIdx.x == 0) {
    // algorithmic bytes, once per group: the entries read under the FP64
    // cut-off, each open member's vectors once
    int open = 0;
    for (int k = 0; k < n; ++k) open += dd_on(G.sysi[k]);
    atomicAdd(ctr, ((unsigned long long)G.entries64 + (unsigned long long)open * 2 * M) * sizeof(cf64));
  }
  for (int k = 0; k < n; ++k) {
    if (!dd_on(G.sysi[k])) continue;
    const cf64* x = G.x[k];
    cf64* P = (cf64*)G.symp[k];
    const cf64 xj = load_x<double>(x, J * kB + c, M);
    // rows of I: V_IJ x_J, real and imaginary parts and the two halves of
    // the wave's rows in separate rounds (register budget: four waves per
    // SIMD)
    constexpr int kH = kRowsPerWave / 2;
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        dd v[kH];
#pragma unroll
        for (int q = 0; q < kH; ++q) {
          const cf64 e = a[half * kH + q];
          v[q] = part == 0 ? two_prod(e.re, xj.re) + (-two_prod(e.im, xj.im))
                           : two_prod(e.re, xj.im) + two_prod(e.im, xj.re);
        }
        wave_reduce_scatter_near<kH>(v, c);
        if (c < kH) {
          const int64_t o = (int64_t)J * ntB + I * kB + w * kRowsPerWave + half * kH +
                            scatter_entry<kH>(c);
          double* ph = reinterpret_cast<double*>(P + o);
          double* pl = reinterpret_cast<double*>(P + np + o);
          ph[part] = v[0].hi;
          pl[part] = v[0].lo;
        }
      }
    if (I != J) {
      // rows of J: V_IJ^T x_I
      const cf64 xi = load_x<double>(x, I * kB + c, M);
      dd cre{0.0, 0.0}, cim{0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kRowsPerWave; ++q) {
        const int r = w * kRowsPerWave + q;
        const double xr = lane_bcast(xi.re, r), xm = lane_bcast(xi.im, r);
        cre += two_prod(a[q].re, xr) + (-two_prod(a[q].im, xm));
        cim += two_prod(a[q].re, xm) + two_prod(a[q].im, xr);
      }
      colred[w][c][0] = cre;
      colred[w][c][1] = cim;
      __syncthreads();
      if (w == 0) {
        const dd ore = (colred[0][c][0] + colred[1][c][0]) + (colred[2][c][0] + colred[3][c][0]);
        const dd oim = (colred[0][c][1] + colred[1][c][1]) + (colred[2][c][1] + colred[3][c][1]);
        const int64_t o = (int64_t)I * ntB + J * kB + c;
        P[o] = cf64{ore.hi, oim.hi};
        P[np + o] = cf64{ore.lo, oim.lo};
      }
      __syncthreads();
    }
  }
}

// r = ghat - sum_Y P[Y][i] in double-double, rounded once (the systems with
// an open outer iteration).
__global__ __launch_bounds__(256) void k_symv_resid_dd_reduce(const SysDesc* __restrict__ sd) {
  const SysDesc D = sd[blockIdx.y];
  if (!D.symp || !dd_on(D.sysi)) return;
  const int M = D.M;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const int nt = sym_blocks(M), ntB = nt * kB;
  const int64_t np = sym_partials(M);
  const cf64* P = (const cf64*)D.symp;
  dd re{D.ghat[i].re, 0.0}, im{D.ghat[i].im, 0.0};
  for (int Y = 0; Y < nt; ++Y) {
    const cf64 h = P[(int64_t)Y * ntB + i], l = P[np + (int64_t)Y * ntB + i];
    re += dd{-h.re, -l.re};
    im += dd{-h.im, -l.im};
  }
  D.r[i] = cf64{re.hi + re.lo, im.hi + im.lo};
}

void launch_resid_dd_groups(const GroupLite* gl, int ngroups, int M, bool grouped,
                            unsigned long long* ctr, hipStream_t s) {
  if (ngroups <= 0) return;
  hipLaunchKernelGGL(k_symv_resid_dd, dim3(sym_tiles(M), ngroups), dim3(256), 0, s, gl,
                     grouped ? 1 : 0, ctr);
  CQM_HIP(hipGetLastError());
}

void launch_resid_dd_reduce(const SysDesc* sd, int nsys, int maxM, hipStream_t s) {
  hipLaunchKernelGGL(k_symv_resid_dd_reduce, dim3((maxM + 255) / 256, nsys), dim3(256), 0, s, sd);
  CQM_HIP(hipGetLastError());
}

template <typename R>
__global__ __launch_bounds__(256) void k_symv_reduce_desc(const SysDesc* __restrict__ sd, int which,
                                                          int j) {
  const SysDesc D = sd[blockIdx.y];
  if (!D.symp) return;  // not a stored-operator system (matrix-free in a mixed batch)
  if (!member_on(D.sysi, which)) return;
  const int M = D.M;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const cplx<R> v = sum_partials<R>((const cplx<R>*)D.symp, M, i);
  if (which == 0) {
    ((cplx<R>*)D.basis)[(int64_t)(j + 1) * M + i] = v;
  } else {
    // the FP64 residual ghat - V x, formed here
    cplx<R> o;
    o.re = (R)D.ghat[i].re - v.re;
    o.im = (R)D.ghat[i].im - v.im;
    ((cplx<R>*)(void*)D.r)[i] = o;
  }
}

template <typename R>
void launch_dense_gemv_groups(const GroupLite* gl, int ngroups, int M, bool grouped, int which,
                              int j, unsigned long long* ctr, hipStream_t s) {
  if (ngroups <= 0) return;
  const dim3 grid(sym_tiles(M), ngroups);
  if (grouped)
    hipLaunchKernelGGL((k_symv_groups<R, true>), grid, dim3(256), 0, s, gl, which, j, ctr);
  else
    hipLaunchKernelGGL((k_symv_groups<R, false>), grid, dim3(256), 0, s, gl, which, j, ctr);
  CQM_HIP(hipGetLastError());
}

template <typename R>
void launch_dense_reduce_desc(const SysDesc* sd, int nsys, int maxM, int which, int j,
                              hipStream_t s) {
  hipLaunchKernelGGL((k_symv_reduce_desc<R>), dim3((maxM + 255) / 256, nsys), dim3(256), 0, s, sd,
                     which, j);
  CQM_HIP(hipGetLastError());
}
// ------------------------------------------------------------------
// Block-Jacobi preconditioner.  The diagonal tile (I, I) of the packed slice
// holds the full kSymB x kSymB block of V(s); its inverse comes from
// Gauss-Jordan elimination without pivoting (s-bar V(s) has a positive
// definite Hermitian part for Re s > 0, so the pivots stay away from zero;
// a vanishing or non-finite pivot leaves the identity for that block).
// Rows and columns past M (the ragged last block) are the identity.
// The block stays in registers: lane c of wave w holds column c of rows
// 16 w .. 16 w + 15.  Step k publishes pivot row k (from its owner wave)
// and each wave's entries of column k (from lane k) through LDS, double
// buffered by the parity of k, so each step has one barrier.
template <typename R>
__global__ __launch_bounds__(256) void k_block_inverse(const cf64* __restrict__ d64, int M,
                                                       int compact, cplx<R>* __restrict__ pinv) {
  // elimination in the precision of the stored inverse (FP32 for the mixed
  // form: half the registers, so every block of a C2 operator is resident
  // at once; the preconditioner only has to be one fixed matrix)
  using Z = cplx<R>;
  __shared__ Z rowb[2][kB];
  __shared__ Z colb[2][4][kRowsPerWave];
  const int I = blockIdx.x, l = blockIdx.y, nb = sym_blocks(M);
  // the diagonal tile of the packed slice, or block I of the compact
  // array of diagonal blocks [frequency][block]
  const cf64* T = compact ? d64 + ((int64_t)l * nb + I) * kB * kB
                          : d64 + (int64_t)l * sym_slice(M) + (int64_t)(I * (I + 1) / 2 + I) * kB * kB;
  const int rows = min(kB, M - I * kB);
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  Z a[kRowsPerWave];
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    const int r = w * kRowsPerWave + q;
    const cf64 v = (r < rows && c < rows) ? T[r * kB + c] : cf64{r == c ? 1.0 : 0.0, 0.0};
    a[q] = cmake<R>((R)v.re, (R)v.im);
  }
  bool bad = false;
  for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
    for (int kq = 0; kq < kRowsPerWave; ++kq) {
      const int k = kb * kRowsPerWave + kq, buf = kq & 1;
      if (w == kb) rowb[buf][c] = a[kq];
      if (c == k) {
#pragma unroll
        for (int q = 0; q < kRowsPerWave; ++q) colb[buf][w][q] = a[q];
      }
      __syncthreads();
      const Z d = rowb[buf][k];
      const R dn = d.re * d.re + d.im * d.im;
      bad |= !(dn > R(0)) || !isfinite(dn);
      const R id = R(1) / dn;
      const Z pk = cmake<R>(d.re * id, -d.im * id);  // 1 / a_kk
      // new pivot row: a_kc / a_kk, and 1 / a_kk at c = k
      const Z rk = rowb[buf][c];
      const Z nr = c == k ? pk : cmake<R>(rk.re * pk.re - rk.im * pk.im, rk.re * pk.im + rk.im * pk.re);
      // rows r != k: a_rc - a_rk a'_kc, and at c = k the new entry
      // -a_rk / a_kk, which is a_rk - a_rk (1 / a_kk + 1): one update form
      // for every lane
      const Z nu = cmake<R>(c == k ? nr.re + R(1) : nr.re, nr.im);
#pragma unroll
      for (int q = 0; q < kRowsPerWave; ++q) {
        const Z ck = colb[buf][w][q];  // a_rk, r = 16 w + q
        a[q].re = fma(-ck.re, nu.re, fma(ck.im, nu.im, a[q].re));
        a[q].im = fma(-ck.re, nu.im, fma(-ck.im, nu.re, a[q].im));
      }
      if (w == kb) a[kq] = nr;
    }
  }
  Z* out = pinv + ((int64_t)l * nb + I) * kB * kB;
#pragma unroll
  for (int q = 0; q < kRowsPerWave; ++q) {
    const int r = w * kRowsPerWave + q;
    out[r * kB + c] = bad ? cmake<R>(r == c ? R(1) : R(0), R(0)) : a[q];
  }
}

// basis[j+1] (or zb) = P basis[j] for systems with an open cycle.  Four
// blocks per workgroup, one wave each.
template <typename R>
__global__ __launch_bounds__(256) void k_block_apply(const SysDesc* __restrict__ sd, int j) {
  __shared__ cplx<R> vb[4][kB];
  const SysDesc D = sd[blockIdx.y];
  if (!D.Pinv || !D.sysi[1]) return;
  const int M = D.M, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + w;
  if (blockIdx.x * 4 * kB >= M) return;
  const bool blk = b * kB < M;  // wave-uniform: this wave's block exists
  const int i = b * kB + lane;
  const cplx<R>* Pb = (const cplx<R>*)D.Pinv + (int64_t)b * kB * kB;
  // FP32 blocks are loaded whole before the vector; FP64 ones in chunks
  constexpr bool kWhole = sizeof(R) == 4;
  cplx<R> p[kWhole ? kB : 1];
  if constexpr (kWhole) {
    if (blk) pblock_load<R>(Pb, lane, p);
  }
  const cplx<R>* v = (const cplx<R>*)D.basis + (int64_t)j * M;
  cplx<R> vi = cmake<R>(R(0), R(0));
  if (i < M) vi = as_global(v)[i];
  vb[w][lane] = vi;
  __syncthreads();
  if (!blk) return;
  R re = R(0), im = R(0);
  if constexpr (kWhole) pblock_acc<R, R>(p, vb[w], re, im);
  else pblock_mul<R, R, 16>(Pb, vb[w], lane, re, im);
  cplx<R>* z = D.zb ? (cplx<R>*)D.zb : (cplx<R>*)D.basis + (int64_t)(j + 1) * M;
  if (i < M) z[i] = cmake<R>(re, im);
}

template <typename R>
void launch_block_inverse(const cf64* d64, int M, int nsys, bool compact, cplx<R>* pinv,
                          hipStream_t s) {
  hipLaunchKernelGGL((k_block_inverse<R>), dim3(sym_blocks(M), nsys), dim3(256), 0, s, d64, M,
                     compact ? 1 : 0, pinv);
  CQM_HIP(hipGetLastError());
}
template <typename R>
void launch_block_apply(const SysDesc* sd, int n, int maxM, int j, hipStream_t s) {
  hipLaunchKernelGGL((k_block_apply<R>), dim3((sym_blocks(maxM) + 3) / 4, n), dim3(256), 0, s, sd,
                     j);
  CQM_HIP(hipGetLastError());
}
template void launch_block_inverse<float>(const cf64*, int, int, bool, cf32*, hipStream_t);
template void launch_block_inverse<double>(const cf64*, int, int, bool, cf64*, hipStream_t);
template void launch_block_apply<float>(const SysDesc*, int, int, int, hipStream_t);
template void launch_block_apply<double>(const SysDesc*, int, int, int, hipStream_t);

template void launch_dense_gemv_groups<float>(const GroupLite*, int, int, bool, int, int,
                                              unsigned long long*, hipStream_t);
template void launch_dense_gemv_groups<double>(const GroupLite*, int, int, bool, int, int,
                                               unsigned long long*, hipStream_t);
template void launch_dense_reduce_desc<float>(const SysDesc*, int, int, int, int, hipStream_t);
template void launch_dense_reduce_desc<double>(const SysDesc*, int, int, int, int, hipStream_t);

template void launch_dense_gemv<float>(const cf32*, int, int, const cf32*, int64_t, cf32*, int64_t,
                                       const int*, cf32*, hipStream_t);
template void launch_dense_gemv<double>(const cf64*, int, int, const cf64*, int64_t, cf64*,
                                        int64_t, const int*, cf64*, hipStream_t);

}  // namespace cqm
