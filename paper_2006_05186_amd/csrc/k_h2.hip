// Product with the compressed operator for every frequency system at once
// (eq. lrfinal): y(l) = sum_near C_b x d_b[l] + U_r [sum_far C_b d_b[l]] U_c^T x.
//   1. upward pass   xhat_c = U_c^T x_c at leaves, E_c'^T xhat_c' upwards
//   2. couplings     yhat_r = sum_{core blocks (r,c)} sum_k d_bk[l] C_bk xhat_c
//   3. downward pass yhat_c' += E_c' yhat_parent
//   4. leaves        y_r = U_r yhat_r + sum_{expanded/near blocks} sum_k d_bk[l] C_bk x_c
// Cluster coefficients are laid out [cluster][mu][l] (l fastest) so that a
// wave reads one matrix entry as a broadcast and consecutive systems as
// coalesced vectors.  R: arithmetic precision; S: storage of the slices.
#include "h2_internal.h"
#include "device_util.h"

namespace cqm {

namespace {
constexpr int kHB = 256;
constexpr int kLC = 32;  // systems per workgroup (grid y splits the systems)
template <typename R> __device__ __forceinline__ void cadd_mul(R& re, R& im, R ar, R ai, R br, R bi) {
  re += ar * br - ai * bi;
  im += ar * bi + ai * br;
}
}  // namespace

// xp[k][l] = x_l[perm[k]]  (cluster order, systems fastest)
template <typename R>
__global__ __launch_bounds__(kHB) void k_h2_gather(const int* __restrict__ perm, int M, int nsys,
                                                   const cplx<R>* __restrict__ x, int64_t xs,
                                                   cplx<R>* __restrict__ xp) {
  const int64_t e = (int64_t)blockIdx.x * kHB + threadIdx.x;
  if (e >= (int64_t)M * nsys) return;
  const int k = (int)(e / nsys), l = (int)(e % nsys);
  xp[e] = x[(int64_t)l * xs + perm[k]];
}
// y_l[perm[k]] = yp[k][l]
template <typename R>
__global__ __launch_bounds__(kHB) void k_h2_scatter(const int* __restrict__ perm, int M, int nsys,
                                                    const cplx<R>* __restrict__ yp,
                                                    cplx<R>* __restrict__ y, int64_t ys) {
  const int64_t e = (int64_t)blockIdx.x * kHB + threadIdx.x;
  if (e >= (int64_t)M * nsys) return;
  const int l = (int)(e / M), k = (int)(e % M);
  y[(int64_t)l * ys + perm[k]] = yp[(int64_t)k * nsys + l];
}

template <typename R, typename U>
__global__ __launch_bounds__(kHB) void k_h2_up_leaf(const int* __restrict__ cl, const int* __restrict__ leaves,
                                                    const int* __restrict__ perm, const U* __restrict__ Uleaf,
                                                    const int64_t* __restrict__ uoff, int P, int nsys,
                                                    const cplx<R>* __restrict__ xp,
                                                    cplx<R>* __restrict__ xhat) {
  const int lf = blockIdx.x, c = leaves[lf];
  const int beg = cl[4 * c], n = cl[4 * c + 1] - beg;
  const U* Ul = Uleaf + uoff[lf];
  cplx<R>* out = xhat + (int64_t)c * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < P * ln; e += kHB) {
    const int mu = e / ln, l = lb + e % ln;
    R re = R(0), im = R(0);
#pragma unroll 8
    for (int i = 0; i < n; ++i) {
      const R u = (R)Ul[(int64_t)i * P + mu];
      const cplx<R> v = xp[(int64_t)(beg + i) * nsys + l];
      re += u * v.re;
      im += u * v.im;
    }
    cplx<R> o;
    o.re = re;
    o.im = im;
    out[(int64_t)mu * nsys + l] = o;
  }
}

// xhat_c = sum_{sons s} E_s^T xhat_s  for the non-leaf clusters of one level
template <typename R, typename U>
__global__ __launch_bounds__(kHB) void k_h2_up(const int* __restrict__ list, const int* __restrict__ sons,
                                               const U* __restrict__ E, int P, int nsys,
                                               cplx<R>* __restrict__ xhat) {
  const int c = list[blockIdx.x];
  const int s0 = sons[2 * c], s1 = sons[2 * c + 1];
  if (s0 < 0) return;
  cplx<R>* out = xhat + (int64_t)c * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < P * ln; e += kHB) {
    const int mu = e / ln, l = lb + e % ln;
    R re = R(0), im = R(0);
    for (int q = 0; q < 2; ++q) {
      const int s = q ? s1 : s0;
      const U* Es = E + (int64_t)s * P * P;
      const cplx<R>* xs_ = xhat + (int64_t)s * P * nsys;
#pragma unroll 8
      for (int lam = 0; lam < P; ++lam) {
        const R w = (R)Es[(int64_t)lam * P + mu];
        const cplx<R> v = xs_[(int64_t)lam * nsys + l];
        re += w * v.re;
        im += w * v.im;
      }
    }
    cplx<R> o;
    o.re = re;
    o.im = im;
    out[(int64_t)mu * nsys + l] = o;
  }
}

// yhat_r = sum over core blocks (r, c): sum_k d_bk[l0+l] C_bk xhat_c  (every cluster)

// yhat_c += E_c yhat_parent for the clusters of one level (top-down)
template <typename R, typename U>
__global__ __launch_bounds__(kHB) void k_h2_down(const int* __restrict__ list, const int* __restrict__ cl,
                                                 const U* __restrict__ E, int P, int nsys,
                                                 cplx<R>* __restrict__ yhat) {
  const int c = list[blockIdx.x];
  const int par = cl[4 * c + 2];
  if (par < 0) return;
  const U* Ec = E + (int64_t)c * P * P;
  const cplx<R>* yp = yhat + (int64_t)par * P * nsys;
  cplx<R>* out = yhat + (int64_t)c * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < P * ln; e += kHB) {
    const int lam = e / ln, l = lb + e % ln;
    const int64_t o = (int64_t)lam * nsys + l;
    R re = out[o].re, im = out[o].im;
#pragma unroll 8
    for (int mu = 0; mu < P; ++mu) {
      const R w = (R)Ec[(int64_t)lam * P + mu];
      const cplx<R> v = yp[(int64_t)mu * nsys + l];
      re += w * v.re;
      im += w * v.im;
    }
    out[o].re = re;
    out[o].im = im;
  }
}

// y at the triangles of one leaf: U_leaf yhat_leaf plus the expanded far and
// near blocks whose row cluster contains the leaf.
template <typename R, typename U>
__global__ __launch_bounds__(kHB) void k_h2_leaf_out(const int* __restrict__ cl,
                                                     const int* __restrict__ leaves,
                                                     const U* __restrict__ Uleaf,
                                                     const int64_t* __restrict__ uoff, int P,
                                                     int nsys, const cplx<R>* __restrict__ yhat,
                                                     cplx<R>* __restrict__ yp) {
  const int lf = blockIdx.x, c = leaves[lf];
  const int beg = cl[4 * c], n = cl[4 * c + 1] - beg;
  const U* Ul = Uleaf + uoff[lf];
  const cplx<R>* yh = yhat + (int64_t)c * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < n * ln; e += kHB) {
    const int i = e / ln, l = lb + e % ln;
    R re = R(0), im = R(0);
#pragma unroll 8
    for (int mu = 0; mu < P; ++mu) {
      const R u = (R)Ul[(int64_t)i * P + mu];
      const cplx<R> v = yh[(int64_t)mu * nsys + l];
      re += u * v.re;
      im += u * v.im;
    }
    cplx<R> o;
    o.re = re;
    o.im = im;
    yp[(int64_t)(beg + i) * nsys + l] = o;
  }
}

size_t h2_apply_scratch_bytes(const H2Operator& h, int nsys) {
  return sizeof(cf64) * h.cl.size() * (size_t)h.p * nsys;
}
size_t h2_perm_scratch_bytes(const H2Operator& h, int nsys) {
  return sizeof(cf64) * h.perm.size() * (size_t)nsys;
}

// ------------------------------------------------------------------
// Block-rank products on the matrix cores: for every output row tile
// (16 rows) and its task list,
//   out[row, l] (+)= sum_tasks sum_t sum_j C_t[row, j] (d_t[l] x[x_row0 + j, l]),
// the contraction of the MACA slices C_t with the cluster vectors scaled by
// the frequency fibres d_t (eq. lrfinal).  One wave owns NF tiles of 16
// frequencies.  The fibre value of the lane's frequency scales the B operand
// (the input block) before each rank term, so consecutive terms accumulate
// into the same four real MFMA chains (re re, im im, re im, im re) with no
// dependence of one term on the result of the last; every kFlush terms the
// chains are added into FP-R accumulators by the vector unit (long MFMA
// chains lose accuracy: over all terms of a row tile the FP32 product's
// error grows sevenfold).  Columns
// are taken 32 at a time so the input block stays in registers across the
// rank terms; the next term's slice entries and fibre values are loaded one
// term ahead.  A workgroup holds as many waves as its frequencies need, up
// to kRankWaves<R>; with a single tile of frequencies (KS > 1) its KS waves
// share the row tile instead, each taking every KS-th task, and their sums
// are added in wave order through LDS.
namespace {
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename R> struct Mfma;
template <> struct Mfma<float> {
  using acc = mf4;
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in element v of lane L
  static __device__ __forceinline__ int row(int L, int v) { return 4 * (L >> 4) + v; }
};
template <> struct Mfma<double> {
  using acc = md4;
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int L, int v) { return (L >> 4) + 4 * v; }
};
constexpr int kKC = 32;  // columns per register block
constexpr int kFlush = 4;  // rank terms per MFMA chain
// waves per workgroup: 4.  Wider workgroups (12 waves for FP32, 8 for FP64)
// cut the FP32 far products' fetched bytes by half but measured no faster
template <typename R> constexpr int kRankWaves = 4;
}  // namespace

template <typename R, typename S, int NF, bool kAccum, int KS>
__global__ __launch_bounds__(64 * kRankWaves<R>) void k_h2_rank_mfma(const RankTile* __restrict__ tiles,
                                                      const RankTask* __restrict__ tasks,
                                                      const int* __restrict__ ranks,
                                                      const cplx<S>* __restrict__ cstore,
                                                      const cf64* __restrict__ dvec, int dstride,
                                                      int l0, int nsys, int ntiles, int gy,
                                                      const cplx<R>* __restrict__ x,
                                                      cplx<R>* __restrict__ out) {
  using MF = Mfma<R>;
  using A4 = typename MF::acc;
  // Workgroups are dealt to the eight dies in turn, so the gy frequency
  // workgroups of one row tile get ids eight apart: they run on one die and
  // read the tile's slices through its L2 once.
  const int grp = blockIdx.x / (8 * gy), rem = blockIdx.x % (8 * gy);
  const int fy = rem >> 3, tile = grp * 8 + (rem & 7);
  if (tile >= ntiles) return;  // padding of the last group; no barrier follows
  const RankTile tl = tiles[tile];
  const int L = threadIdx.x & 63, w = threadIdx.x >> 6;
  // first frequency of this wave
  const int fb = KS > 1 ? 0 : (fy * (blockDim.x >> 6) + w) * 16 * NF;
  if (fb >= nsys) return;  // KS == 1 only: no barrier follows
  const int arow = L & 15, kq = L >> 4, col = L & 15;
  const bool rowin = arow < tl.nrows;
  // sums of Cr Br, Ci Bi, Cr Bi, Ci Br over the last terms; acc: the rest
  A4 p1[NF], p2[NF], p3[NF], p4[NF], accr[NF], acci[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) p1[f] = p2[f] = p3[f] = p4[f] = accr[f] = acci[f] = MF::zero();
  int chain = 0;
  auto flush = [&]() {
#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        accr[f][v] += p1[f][v] - p2[f][v];
        acci[f][v] += p3[f][v] + p4[f][v];
      }
      p1[f] = p2[f] = p3[f] = p4[f] = MF::zero();
    }
    chain = 0;
  };
  for (int q = tl.t0 + (KS > 1 ? w : 0); q < tl.t1; q += KS) {
    const RankTask T = tasks[q];
    const int rk = ranks[T.block];
    for (int j0 = 0; j0 < T.acols; j0 += kKC) {
      const int nk = min(kKC, T.acols - j0);
      const int ks = (nk + 3) >> 2;
      // input block: x[x_row0 + j0 + 4s + kq, fb + 16 f + col].  Loads use
      // clamped (in-bounds) indices and are masked afterwards, so that they
      // are all in flight together instead of one branch at a time.
      R xr[kKC / 4][NF], xi[kKC / 4][NF];
#pragma unroll
      for (int s = 0; s < kKC / 4; ++s)
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const int j = 4 * s + kq, l = fb + 16 * f + col;
          const bool in = j < nk && l < nsys;
          const cplx<R> v =
              x[(int64_t)(T.x_row0 + j0 + min(j, nk - 1)) * nsys + min(l, nsys - 1)];
          xr[s][f] = in ? v.re : R(0);
          xi[s][f] = in ? v.im : R(0);
        }
      // slice entries and fibre values of rank term t
      const cplx<S>* C0 = cstore + T.c_off + (int64_t)min(arow, tl.nrows - 1) * T.ldc + j0;
      const cf64* D0 = dvec + T.d_off + l0;
      R ar[kKC / 4], ai[kKC / 4], dr[NF], di[NF];
      auto load_term = [&](int t, R* re, R* im, R* fr, R* fi) {
        const int tc = min(t, max(rk - 1, 0));
        const cplx<S>* Cr = C0 + (int64_t)tc * T.cstride;
#pragma unroll
        for (int s = 0; s < kKC / 4; ++s) {
          const int j = 4 * s + kq;
          const bool in = rowin && j < nk;
          const cplx<S> c = Cr[min(j, nk - 1)];
          re[s] = in ? (R)c.re : R(0);
          im[s] = in ? (R)c.im : R(0);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const int l = fb + 16 * f + col;
          const cf64 d = D0[(int64_t)tc * dstride + min(l, nsys - 1)];
          fr[f] = (R)d.re;
          fi[f] = (R)d.im;
        }
      };
      load_term(0, ar, ai, dr, di);
      for (int t = 0; t < rk; ++t) {
        R br[kKC / 4], bi[kKC / 4], er[NF], ei[NF];
        load_term(t + 1, br, bi, er, ei);
#pragma unroll
        for (int s = 0; s < kKC / 4; ++s) {
          if (s < ks) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              const R yr = dr[f] * xr[s][f] - di[f] * xi[s][f];
              const R yi = dr[f] * xi[s][f] + di[f] * xr[s][f];
              p1[f] = MF::mac(ar[s], yr, p1[f]);
              p2[f] = MF::mac(ai[s], yi, p2[f]);
              p3[f] = MF::mac(ar[s], yi, p3[f]);
              p4[f] = MF::mac(ai[s], yr, p4[f]);
            }
          }
        }
#pragma unroll
        for (int s = 0; s < kKC / 4; ++s) {
          ar[s] = br[s];
          ai[s] = bi[s];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          dr[f] = er[f];
          di[f] = ei[f];
        }
        if (++chain == kFlush) flush();
      }
    }
  }
  flush();
  if constexpr (KS > 1) {
    // waves 1 .. KS-1 hand their sums to wave 0, which adds them in order
    __shared__ R red[KS - 1][2 * 4 * NF][64];
    if (w > 0)
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          red[w - 1][8 * f + v][L] = accr[f][v];
          red[w - 1][8 * f + 4 + v][L] = acci[f][v];
        }
    __syncthreads();
    if (w > 0) return;
    for (int u = 0; u < KS - 1; ++u)
#pragma unroll
      for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          accr[f][v] += red[u][8 * f + v][L];
          acci[f][v] += red[u][8 * f + 4 + v][L];
        }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = MF::row(L, v), l = fb + 16 * f + col;
      if (i < tl.nrows && l < nsys) {
        cplx<R>* o = out + (int64_t)(tl.out_row0 + i) * nsys + l;
        cplx<R> r;
        r.re = accr[f][v];
        r.im = acci[f][v];
        if (kAccum) {
          const cplx<R> e = *o;
          r.re += e.re;
          r.im += e.im;
        }
        *o = r;
      }
    }
}

template <typename R, typename S, bool kAccum>
static void launch_rank_mfma(const RankTile* tiles, int ntiles, const RankTask* tasks,
                             const int* ranks, const void* cstore, const cf64* dvec, int dstride,
                             int l0, int nsys, const cplx<R>* x, cplx<R>* out, hipStream_t s) {
  if (ntiles <= 0) return;
  constexpr int NF = 1;
  // 16 NF frequencies per wave; the fewest workgroups per row tile, with the
  // waves spread evenly over them.  One tile of frequencies: the row tile's
  // tasks split over kRankWaves<R> waves of one workgroup.
  const int ftiles = (nsys + 16 * NF - 1) / (16 * NF);
  if (ftiles == 1) {
    constexpr int KS = kRankWaves<R>;
    const dim3 grid((unsigned)(((ntiles + 7) / 8) * 8));
    hipLaunchKernelGGL((k_h2_rank_mfma<R, S, NF, kAccum, KS>), grid, dim3(64 * KS), 0, s, tiles, tasks,
                       ranks, (const cplx<S>*)cstore, dvec, dstride, l0, nsys, ntiles, 1, x, out);
    CQM_HIP(hipGetLastError());
    return;
  }
  const int gy = (ftiles + kRankWaves<R> - 1) / kRankWaves<R>;
  const int nw = (ftiles + gy - 1) / gy;
  const dim3 grid((unsigned)(((ntiles + 7) / 8) * 8 * gy));
  hipLaunchKernelGGL((k_h2_rank_mfma<R, S, NF, kAccum, 1>), grid, dim3(64 * nw), 0, s, tiles, tasks, ranks,
                     (const cplx<S>*)cstore, dvec, dstride, l0, nsys, ntiles, gy, x, out);
  CQM_HIP(hipGetLastError());
}

// The slices, ranks and fibres a product contracts: the operator's own, or
// the collapsed lag-0 slices of the time-marching weights.
struct RankOperands {
  const RankTask* core_tasks;
  const RankTask* leaf_tasks;
  const int* ranks;
  const void* cstore;
  const cf64* dvec;
  int dstride;
};

template <typename R>
static void h2_apply_with(const Problem& p, H2Operator& h, const RankOperands& op, int l0, int nsys,
                          const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys, hipStream_t s) {
  const cf64* dv = op.dvec;
  const int P = h.p;
  cplx<R>* xh = (cplx<R>*)h.xhat_d;
  cplx<R>* yh = (cplx<R>*)h.yhat_d;
  const int nleaf = (int)h.leaves.size();
  const bool f32 = sizeof(R) == 4;
  const int dstride = op.dstride;
  const int M = (int)h.perm.size();
  cplx<R>* xp = (cplx<R>*)h.xp_d;
  cplx<R>* yp = (cplx<R>*)h.yp_d;
  const unsigned gblk = (unsigned)(((int64_t)M * nsys + kHB - 1) / kHB);
  const int nch = (nsys + kLC - 1) / kLC;
  hipLaunchKernelGGL((k_h2_gather<R>), dim3(gblk), dim3(kHB), 0, s, h.perm_d, M, nsys, x, xs, xp);
  if (h.n_core == 0) {
    // no block kept as a Tucker core (every admissible block small enough
    // to be expanded): no cluster coefficients, the leaf products write y
    if (h.store_fp64)
      launch_rank_mfma<R, double, false>(h.leaf_tiles_d, h.n_leaf_tiles, op.leaf_tasks, op.ranks,
                                         op.cstore, dv, dstride, l0, nsys, xp, yp, s);
    else
      launch_rank_mfma<R, float, false>(h.leaf_tiles_d, h.n_leaf_tiles, op.leaf_tasks, op.ranks,
                                        op.cstore, dv, dstride, l0, nsys, xp, yp, s);
    hipLaunchKernelGGL((k_h2_scatter<R>), dim3(gblk), dim3(kHB), 0, s, h.perm_d, M, nsys, yp, y, ys);
    CQM_HIP(hipGetLastError());
    return;
  }
  // 1. upward pass
  if (f32)
    hipLaunchKernelGGL((k_h2_up_leaf<R, float>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, h.level_cl_d + h.level_off[h.nlevels],
                       h.perm_d, h.U32_d, h.uleaf_off_d, P, nsys, xp, xh);
  else
    hipLaunchKernelGGL((k_h2_up_leaf<R, double>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, h.level_cl_d + h.level_off[h.nlevels],
                       h.perm_d, h.U_d, h.uleaf_off_d, P, nsys, xp, xh);
  CQM_HIP(hipGetLastError());
  for (int lv = h.nlevels - 2; lv >= 0; --lv) {
    const int cnt = h.level_off[lv + 1] - h.level_off[lv];
    if (f32)
      hipLaunchKernelGGL((k_h2_up<R, float>), dim3(cnt, nch), dim3(kHB), 0, s, h.level_cl_d + h.level_off[lv],
                         h.cl_d + 4 * (int)h.cl.size(), h.E32_d, P, nsys, xh);
    else
      hipLaunchKernelGGL((k_h2_up<R, double>), dim3(cnt, nch), dim3(kHB), 0, s, h.level_cl_d + h.level_off[lv],
                         h.cl_d + 4 * (int)h.cl.size(), h.E_d, P, nsys, xh);
    CQM_HIP(hipGetLastError());
  }
  // 2. couplings: every cluster's coefficient rows (zero where no core block)
  if (h.store_fp64)
    launch_rank_mfma<R, double, false>(h.core_tiles_d, h.n_core_tiles, op.core_tasks, op.ranks,
                                       op.cstore, dv, dstride, l0, nsys, xh, yh, s);
  else
    launch_rank_mfma<R, float, false>(h.core_tiles_d, h.n_core_tiles, op.core_tasks, op.ranks,
                                      op.cstore, dv, dstride, l0, nsys, xh, yh, s);
  // 3. downward pass
  for (int lv = 1; lv < h.nlevels; ++lv) {
    const int cnt = h.level_off[lv + 1] - h.level_off[lv];
    if (f32)
      hipLaunchKernelGGL((k_h2_down<R, float>), dim3(cnt, nch), dim3(kHB), 0, s, h.level_cl_d + h.level_off[lv], h.cl_d,
                         h.E32_d, P, nsys, yh);
    else
      hipLaunchKernelGGL((k_h2_down<R, double>), dim3(cnt, nch), dim3(kHB), 0, s, h.level_cl_d + h.level_off[lv], h.cl_d,
                         h.E_d, P, nsys, yh);
    CQM_HIP(hipGetLastError());
  }
  // 4. leaves: y_r = U_r yhat_r, then the expanded-far and near blocks
  const int* lvs = h.level_cl_d + h.level_off[h.nlevels];
  if (f32)
    hipLaunchKernelGGL((k_h2_leaf_out<R, float>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs,
                       h.U32_d, h.uleaf_off_d, P, nsys, yh, yp);
  else
    hipLaunchKernelGGL((k_h2_leaf_out<R, double>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs,
                       h.U_d, h.uleaf_off_d, P, nsys, yh, yp);
  CQM_HIP(hipGetLastError());
  if (h.store_fp64)
    launch_rank_mfma<R, double, true>(h.leaf_tiles_d, h.n_leaf_tiles, op.leaf_tasks, op.ranks,
                                      op.cstore, dv, dstride, l0, nsys, xp, yp, s);
  else
    launch_rank_mfma<R, float, true>(h.leaf_tiles_d, h.n_leaf_tiles, op.leaf_tasks, op.ranks,
                                     op.cstore, dv, dstride, l0, nsys, xp, yp, s);
  hipLaunchKernelGGL((k_h2_scatter<R>), dim3(gblk), dim3(kHB), 0, s, h.perm_d, M, nsys, yp, y, ys);
  CQM_HIP(hipGetLastError());
}

template <typename R>
void launch_h2_apply(const Problem& p, H2Operator& h, int l0, int nsys, const cplx<R>* x, int64_t xs,
                     cplx<R>* y, int64_t ys, const cf64* fibres, hipStream_t s) {
  // the frequency fibres d_t[l], or their transforms (time-marching weights)
  const RankOperands op{h.core_tasks_d, h.leaf_tasks_d, h.ranks_d, h.cstore_d,
                        fibres ? fibres : h.dvec_d, h.nsys};
  h2_apply_with<R>(p, h, op, l0, nsys, x, xs, y, ys, s);
}

// What_0 = Re W0 written densely (triangle order, row-major M x M, FP64).
// One workgroup per block: near and expanded far blocks copy the real part
// of their collapsed slice; a core forms T = U_r Re(W0_b) a few rows at a
// time in LDS, then T U_c^T (full cluster bases).  The blocks partition the
// matrix, so every entry is written once.
constexpr int kExpandLds = 2048;
template <typename S>
__global__ __launch_bounds__(256) void k_expand_lag0(const BlockDesc* __restrict__ blocks, int Rcap,
                                                     const cplx<S>* __restrict__ w0,
                                                     const int* __restrict__ cl,
                                                     const int* __restrict__ perm,
                                                     const double* __restrict__ Ufull,
                                                     const int64_t* __restrict__ uoff, int P, int M,
                                                     double* __restrict__ W) {
  const BlockDesc B = blocks[blockIdx.x];
  const int rb = cl[4 * B.r], cb = cl[4 * B.c];
  const cplx<S>* C = w0 + B.c_off / Rcap;
  if (B.kind != kFarCore) {
    const int n = B.arows * B.acols;
    for (int e = threadIdx.x; e < n; e += 256) {
      const int i = e / B.acols, j = e - i * B.acols;
      W[(int64_t)perm[rb + i] * M + perm[cb + j]] = (double)C[e].re;
    }
    return;
  }
  __shared__ double Tsh[kExpandLds];
  const int rows = cl[4 * B.r + 1] - rb, cols = cl[4 * B.c + 1] - cb;
  const double* Ur = Ufull + uoff[B.r];
  const double* Uc = Ufull + uoff[B.c];
  const int rows_per = max(1, kExpandLds / P);
  for (int i0 = 0; i0 < rows; i0 += rows_per) {
    const int nr = min(rows_per, rows - i0);
    for (int e = threadIdx.x; e < nr * P; e += 256) {
      const int i = i0 + e / P, nu = e % P;
      double acc = 0.0;
      for (int mu = 0; mu < P; ++mu) acc += Ur[(int64_t)i * P + mu] * (double)C[(int64_t)mu * P + nu].re;
      Tsh[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * cols; e += 256) {
      const int ii = e / cols, j = e - ii * cols;
      double acc = 0.0;
      for (int nu = 0; nu < P; ++nu) acc += Tsh[ii * P + nu] * Uc[(int64_t)j * P + nu];
      W[(int64_t)perm[rb + i0 + ii] * M + perm[cb + j]] = acc;
    }
    __syncthreads();
  }
}

void launch_expand_lag0(const Problem& p, H2Operator& h, hipStream_t s) {
  require(h.p <= kExpandLds, CQM_EINVAL, "interpolation rank above the expansion tile");
  const unsigned nb = (unsigned)h.blocks.size();
  const int M = (int)h.perm.size();
  if (nb == 0) return;
  if (h.store_fp64)
    hipLaunchKernelGGL((k_expand_lag0<double>), dim3(nb), dim3(256), 0, s, h.blocks_d, h.Rcap,
                       (const cf64*)h.w0_d, h.cl_d, h.perm_d, h.Ufull_d, h.ufull_off_d, h.p, M,
                       h.w0dense_d);
  else
    hipLaunchKernelGGL((k_expand_lag0<float>), dim3(nb), dim3(256), 0, s, h.blocks_d, h.Rcap,
                       (const cf32*)h.w0_d, h.cl_d, h.perm_d, h.Ufull_d, h.ufull_off_d, h.p, M,
                       h.w0dense_d);
  CQM_HIP(hipGetLastError());
}

// y = What_0 q for the real parts of q: one wave per row, lanes along the
// row (coalesced), the row sum in a fixed order; y's imaginary part is 0.
__global__ __launch_bounds__(256) void k_lag0_dense_product(const double* __restrict__ W, int M,
                                                            const cf64* __restrict__ q,
                                                            cf64* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= M) return;  // whole waves leave: no barrier follows
  const double* w = W + (int64_t)row * M;
  double acc = 0.0;
#pragma unroll 4
  for (int j = lane; j < M; j += 64) acc += w[j] * q[j].re;
  acc = wave_sum(acc);
  if (lane == 0) y[row] = cf64{acc, 0.0};
}

void launch_lag0_dense_product(const H2Operator& h, const cf64* q, cf64* y, hipStream_t s) {
  const int M = (int)h.perm.size();
  hipLaunchKernelGGL(k_lag0_dense_product, dim3((M + 3) / 4), dim3(256), 0, s, h.w0dense_d, M, q, y);
  CQM_HIP(hipGetLastError());
}

// W0_b[e] = sum_{t < rank_b} dhat_t[0] C_t[e]: one workgroup per block, the
// block's lag-0 fibre values staged in LDS, FP64 sums rounded once.
constexpr int kCollapseMaxR = 128;
template <typename S>
__global__ __launch_bounds__(256) void k_collapse_lag0(const BlockDesc* __restrict__ blocks,
                                                       const int* __restrict__ ranks,
                                                       const cplx<S>* __restrict__ cstore,
                                                       const cf64* __restrict__ dhat, int nsys,
                                                       int Rcap, cplx<S>* __restrict__ w0) {
  __shared__ cf64 d0[kCollapseMaxR];
  const BlockDesc B = blocks[blockIdx.x];
  const int rk = ranks[blockIdx.x];
  for (int t = threadIdx.x; t < rk; t += 256) d0[t] = dhat[B.d_off + (int64_t)t * nsys];
  __syncthreads();
  const int64_t n = (int64_t)B.arows * B.acols;
  const cplx<S>* C = cstore + B.c_off;
  cplx<S>* W = w0 + B.c_off / Rcap;
  for (int64_t e = threadIdx.x; e < n; e += 256) {
    double re = 0.0, im = 0.0;
    for (int t = 0; t < rk; ++t) {
      const cplx<S> c = C[(int64_t)t * n + e];
      const cf64 d = d0[t];
      re += d.re * (double)c.re - d.im * (double)c.im;
      im += d.re * (double)c.im + d.im * (double)c.re;
    }
    cplx<S> v;
    v.re = (S)re;
    v.im = (S)im;
    W[e] = v;
  }
}

void launch_collapse_lag0(const Problem& p, H2Operator& h, hipStream_t s) {
  require(h.Rcap <= kCollapseMaxR, CQM_EINVAL, "rank cap above the lag-0 collapse limit");
  const unsigned nb = (unsigned)h.blocks.size();
  if (nb == 0) return;
  if (h.store_fp64)
    hipLaunchKernelGGL((k_collapse_lag0<double>), dim3(nb), dim3(256), 0, s, h.blocks_d, h.ranks_d,
                       (const cf64*)h.cstore_d, h.dhat_d, h.nsys, h.Rcap, (cf64*)h.w0_d);
  else
    hipLaunchKernelGGL((k_collapse_lag0<float>), dim3(nb), dim3(256), 0, s, h.blocks_d, h.ranks_d,
                       (const cf32*)h.cstore_d, h.dhat_d, h.nsys, h.Rcap, (cf32*)h.w0_d);
  CQM_HIP(hipGetLastError());
}

// ------------------------------------------------------------------
// Fast right-hand side of the compressed marching (eq. fastrhs):
//   sum_{k=1}^{n} What_k x_{n-k} = sum_b sum_t C_bt (sum_k dhat_bt[k] x_{n-k}|cols b)
// The inner sums (the fibres convolved with the block's column history) are
// formed first, then one product per block and rank term: one pass over
// the slices per step instead of one per lag.

// z_{b,t}[j] = sum_{k=1}^{n} dhat_bt[k] h_{n-k}[col_b + j]; h: past inputs in
// cluster order (expanded far and near blocks) or their cluster
// coefficients (cores).  One workgroup per block.
__global__ __launch_bounds__(256) void k_fast_conv(const BlockDesc* __restrict__ blocks,
                                                   const int* __restrict__ ranks,
                                                   const int64_t* __restrict__ zoff,
                                                   const int* __restrict__ cl, int P,
                                                   const cf64* __restrict__ dhat, int F, int n,
                                                   const cf64* __restrict__ hx, int64_t sx,
                                                   const cf64* __restrict__ hxh, int64_t sxh,
                                                   cf64* __restrict__ z) {
  const int b = blockIdx.x;
  const BlockDesc B = blocks[b];
  const int rk = ranks[b], nc = B.acols;
  const bool core = B.kind == kFarCore;
  const cf64* H = core ? hxh + (int64_t)B.c * P : hx + cl[4 * B.c];
  const int64_t sh = core ? sxh : sx;
  cf64* zb = z + zoff[b];
  for (int e = threadIdx.x; e < rk * nc; e += 256) {
    const int t = e / nc, j = e - t * nc;
    const cf64* d = dhat + B.d_off + (int64_t)t * F;
    double re = 0.0, im = 0.0;
#pragma unroll 4
    for (int k = 1; k <= n; ++k) {
      const cf64 a = d[k], v = H[(int64_t)(n - k) * sh + j];
      re += a.re * v.re - a.im * v.im;
      im += a.re * v.im + a.im * v.re;
    }
    zb[e] = cf64{re, im};
  }
}

// One system, split K: part[y][out_row0 + row] = sum over the tasks
// q = t0 + y, t0 + y + kConvSplit, .. of the row tile and their rank terms of
// C_t[row, :] . z_{b,t}.  Sixteen lanes per row take every sixteenth column;
// their sums are combined by a fixed butterfly.
template <typename S>
__global__ __launch_bounds__(256) void k_h2_rank_conv(const RankTile* __restrict__ tiles,
                                                      const RankTask* __restrict__ tasks,
                                                      const int* __restrict__ ranks,
                                                      const int64_t* __restrict__ zoff,
                                                      const cplx<S>* __restrict__ cstore,
                                                      const cf64* __restrict__ z, int64_t pstride,
                                                      cf64* __restrict__ part) {
  const RankTile tl = tiles[blockIdx.x];
  const int y = blockIdx.y;
  const int row = threadIdx.x >> 4, lane = threadIdx.x & 15;
  double re = 0.0, im = 0.0;
  if (row < tl.nrows) {
    for (int q = tl.t0 + y; q < tl.t1; q += kConvSplit) {
      const RankTask T = tasks[q];
      const int rk = ranks[T.block];
      const cplx<S>* Crow = cstore + T.c_off + (int64_t)row * T.ldc;
      const cf64* zt = z + zoff[T.block];
      for (int t = 0; t < rk; ++t) {
        const cplx<S>* Ct = Crow + (int64_t)t * T.cstride;
        const cf64* zz = zt + (int64_t)t * T.acols;
        for (int j = lane; j < T.acols; j += 16) {
          const cplx<S> c = Ct[j];
          const cf64 v = zz[j];
          re += (double)c.re * v.re - (double)c.im * v.im;
          im += (double)c.re * v.im + (double)c.im * v.re;
        }
      }
    }
  }
  for (int off = 8; off > 0; off >>= 1) {
    re += __shfl_xor(re, off, 16);
    im += __shfl_xor(im, off, 16);
  }
  if (lane == 0 && row < tl.nrows) part[(int64_t)y * pstride + tl.out_row0 + row] = cf64{re, im};
}

// out[i] (+)= sum_{y < kConvSplit} part[y][i], in order of y
template <bool kAccum>
__global__ __launch_bounds__(256) void k_conv_reduce(const cf64* __restrict__ part, int64_t pstride,
                                                     int64_t n, cf64* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  for (int y = 0; y < kConvSplit; ++y) {
    const cf64 v = part[(int64_t)y * pstride + i];
    re += v.re;
    im += v.im;
  }
  if (kAccum) {
    out[i].re += re;
    out[i].im += im;
  } else {
    out[i] = cf64{re, im};
  }
}

static void conv_products(const H2Operator& h, const RankTile* tiles, int ntiles,
                          const RankTask* tasks, int64_t rows, bool accum, cf64* out,
                          hipStream_t s) {
  if (ntiles <= 0) return;
  const int64_t ps = (int64_t)std::max(h.cl.size() * (size_t)h.p, h.perm.size());
  const dim3 grid((unsigned)ntiles, kConvSplit);
  if (h.store_fp64)
    hipLaunchKernelGGL((k_h2_rank_conv<double>), grid, dim3(256), 0, s, tiles, tasks, h.ranks_d,
                       h.zoff_d, (const cf64*)h.cstore_d, h.z_d, ps, h.rpart_d);
  else
    hipLaunchKernelGGL((k_h2_rank_conv<float>), grid, dim3(256), 0, s, tiles, tasks, h.ranks_d,
                       h.zoff_d, (const cf32*)h.cstore_d, h.z_d, ps, h.rpart_d);
  CQM_HIP(hipGetLastError());
  const unsigned g = (unsigned)((rows + 255) / 256);
  if (accum)
    hipLaunchKernelGGL((k_conv_reduce<true>), dim3(g), dim3(256), 0, s, h.rpart_d, ps, rows, out);
  else
    hipLaunchKernelGGL((k_conv_reduce<false>), dim3(g), dim3(256), 0, s, h.rpart_d, ps, rows, out);
  CQM_HIP(hipGetLastError());
}

void launch_h2_push_history(const Problem& p, H2Operator& h, int m, const cf64* x, cf64* hx,
                            hipStream_t s) {
  const int M = (int)h.perm.size(), P = h.p, nleaf = (int)h.leaves.size();
  require(m >= 0 && m < p.F, CQM_EINVAL, "history slot out of range");
  hipLaunchKernelGGL((k_h2_gather<double>), dim3((M + kHB - 1) / kHB), dim3(kHB), 0, s, h.perm_d, M, 1,
                     x, (int64_t)M, hx);
  CQM_HIP(hipGetLastError());
  if (h.n_core == 0) return;
  cf64* xh = h.hxh_d + (int64_t)m * h.cl.size() * P;
  hipLaunchKernelGGL((k_h2_up_leaf<double, double>), dim3(nleaf, 1), dim3(kHB), 0, s, h.cl_d,
                     h.level_cl_d + h.level_off[h.nlevels], h.perm_d, h.U_d, h.uleaf_off_d, P, 1, hx, xh);
  CQM_HIP(hipGetLastError());
  for (int lv = h.nlevels - 2; lv >= 0; --lv) {
    const int cnt = h.level_off[lv + 1] - h.level_off[lv];
    hipLaunchKernelGGL((k_h2_up<double, double>), dim3(cnt, 1), dim3(kHB), 0, s,
                       h.level_cl_d + h.level_off[lv], h.cl_d + 4 * (int)h.cl.size(), h.E_d, P, 1, xh);
    CQM_HIP(hipGetLastError());
  }
}

void launch_h2_fast_history(const Problem& p, H2Operator& h, int n, const cf64* hx, cf64* y,
                            hipStream_t s) {
  const int M = (int)h.perm.size(), P = h.p, nleaf = (int)h.leaves.size();
  require(n >= 1 && n < p.F && h.nsys == p.F, CQM_EINVAL, "history length out of range");
  const int nb = (int)h.blocks.size();
  const int64_t coef = (int64_t)h.cl.size() * P;
  if (nb > 0) {
    hipLaunchKernelGGL(k_fast_conv, dim3(nb), dim3(256), 0, s, h.blocks_d, h.ranks_d, h.zoff_d, h.cl_d, P,
                       h.dhat_d, h.nsys, n, hx, (int64_t)M, h.hxh_d, coef, h.z_d);
    CQM_HIP(hipGetLastError());
  }
  cf64* yh = (cf64*)h.yhat_d;
  cf64* yp = (cf64*)h.yp_d;
  if (h.n_core > 0) {
    conv_products(h, h.core_tiles_d, h.n_core_tiles, h.core_tasks_d, coef, false, yh, s);
    for (int lv = 1; lv < h.nlevels; ++lv) {
      const int cnt = h.level_off[lv + 1] - h.level_off[lv];
      hipLaunchKernelGGL((k_h2_down<double, double>), dim3(cnt, 1), dim3(kHB), 0, s,
                         h.level_cl_d + h.level_off[lv], h.cl_d, h.E_d, P, 1, yh);
      CQM_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL((k_h2_leaf_out<double, double>), dim3(nleaf, 1), dim3(kHB), 0, s, h.cl_d,
                       h.level_cl_d + h.level_off[h.nlevels], h.U_d, h.uleaf_off_d, P, 1, yh, yp);
    CQM_HIP(hipGetLastError());
    conv_products(h, h.leaf_tiles_d, h.n_leaf_tiles, h.leaf_tasks_d, M, true, yp, s);
  } else {
    conv_products(h, h.leaf_tiles_d, h.n_leaf_tiles, h.leaf_tasks_d, M, false, yp, s);
  }
  hipLaunchKernelGGL((k_h2_scatter<double>), dim3((M + kHB - 1) / kHB), dim3(kHB), 0, s, h.perm_d, M, 1,
                     yp, y, (int64_t)M);
  CQM_HIP(hipGetLastError());
}

template void launch_h2_apply<float>(const Problem&, H2Operator&, int, int, const cf32*, int64_t, cf32*,
                                     int64_t, const cf64*, hipStream_t);
template void launch_h2_apply<double>(const Problem&, H2Operator&, int, int, const cf64*, int64_t, cf64*,
                                      int64_t, const cf64*, hipStream_t);

// One thread per (fibre slot, n): dhat[n] = rho^-n / F sum_l d[l] zeta^(n l mod F)
// (twiddles and scales from the problem's tables; the index n l mod F is
// carried incrementally).
__global__ __launch_bounds__(256) void k_fibre_dft(const cf64* __restrict__ d, int64_t slots, int F,
                                                   const cf64* __restrict__ tw,
                                                   const double* __restrict__ scale,
                                                   cf64* __restrict__ dhat) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= slots * F) return;
  const int64_t slot = g / F;
  const int n = (int)(g - slot * F);
  const cf64* ds = d + slot * F;
  double re = 0.0, im = 0.0;
  int k = 0;
  for (int l = 0; l < F; ++l) {
    const cf64 a = ds[l], t = tw[k];
    re += a.re * t.re - a.im * t.im;
    im += a.re * t.im + a.im * t.re;
    k += n;
    if (k >= F) k -= F;
  }
  dhat[g] = cf64{re * scale[n], im * scale[n]};
}

void launch_fibre_dft(const Problem& p, const H2Operator& h, const cf64* d, cf64* dhat, hipStream_t s) {
  require(h.nsys == p.F, CQM_EINVAL, "the fibre transform needs the full band of frequencies");
  const int64_t slots = h.dvec_elems / p.F;
  const int64_t n = slots * p.F;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fibre_dft, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, slots, p.F,
                     p.dev.tw_inv, p.dev.rho_ipow, dhat);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
