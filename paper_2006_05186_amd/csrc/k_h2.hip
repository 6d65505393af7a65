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
template <typename R, typename S>
__global__ __launch_bounds__(kHB) void k_h2_couple(const int* __restrict__ rowptr, const int* __restrict__ list,
                                                   const BlockDesc* __restrict__ blocks,
                                                   const int* __restrict__ ranks,
                                                   const cplx<S>* __restrict__ cstore,
                                                   const cf64* __restrict__ dvec, int dstride, int l0,
                                                   int P, int nsys, const cplx<R>* __restrict__ xhat,
                                                   cplx<R>* __restrict__ yhat) {
  const int r = blockIdx.x;
  cplx<R>* out = yhat + (int64_t)r * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < P * ln; e += kHB) {
    const int mu = e / ln, l = lb + e % ln;
    R re = R(0), im = R(0);
    for (int q = rowptr[r]; q < rowptr[r + 1]; ++q) {
      const int b = list[q];
      const BlockDesc B = blocks[b];
      const cplx<R>* xc = xhat + (int64_t)B.c * P * nsys;
      const int rk = ranks[b];
      for (int t = 0; t < rk; ++t) {
        const cplx<S>* Ct = cstore + B.c_off + (int64_t)t * P * P + (int64_t)mu * P;
        R sr = R(0), si = R(0);
        for (int nu = 0; nu < P; ++nu) {
          const cplx<S> c = Ct[nu];
          const cplx<R> v = xc[(int64_t)nu * nsys + l];
          cadd_mul<R>(sr, si, (R)c.re, (R)c.im, v.re, v.im);
        }
        const cf64 dv = dvec[B.d_off + (int64_t)t * dstride + l0 + l];
        cadd_mul<R>(re, im, (R)dv.re, (R)dv.im, sr, si);
      }
    }
    cplx<R> o;
    o.re = re;
    o.im = im;
    out[(int64_t)mu * nsys + l] = o;
  }
}

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
template <typename R, typename S, typename U>
__global__ __launch_bounds__(kHB) void k_h2_leaf_out(
    const int* __restrict__ cl, const int* __restrict__ leaves, const int* __restrict__ perm,
    const U* __restrict__ Uleaf, const int64_t* __restrict__ uoff, int P, int nsys,
    const cplx<R>* __restrict__ yhat, const int* __restrict__ trow, const LeafTask* __restrict__ tasks,
    const BlockDesc* __restrict__ blocks, const int* __restrict__ ranks,
    const cplx<S>* __restrict__ cstore, const cf64* __restrict__ dvec, int dstride, int l0,
    const cplx<R>* __restrict__ xp, cplx<R>* __restrict__ yp) {
  const int lf = blockIdx.x, c = leaves[lf];
  const int beg = cl[4 * c], n = cl[4 * c + 1] - beg;
  const U* Ul = Uleaf + uoff[lf];
  const cplx<R>* yh = yhat + (int64_t)c * P * nsys;
  const int lb = blockIdx.y * kLC, ln = min(kLC, nsys - lb);
  for (int e = threadIdx.x; e < n * ln; e += kHB) {
    const int i = e / ln, l = lb + e % ln;
    R re = R(0), im = R(0);
    for (int mu = 0; mu < P; ++mu) {
      const R u = (R)Ul[(int64_t)i * P + mu];
      const cplx<R> v = yh[(int64_t)mu * nsys + l];
      re += u * v.re;
      im += u * v.im;
    }
    for (int q = trow[lf]; q < trow[lf + 1]; ++q) {
      const LeafTask T = tasks[q];
      const BlockDesc B = blocks[T.block];
      const int cb = cl[4 * B.c];
      const int rk = ranks[T.block];
      const int row = T.rowoff + i;
      for (int t = 0; t < rk; ++t) {
        const cplx<S>* Ct = cstore + B.c_off + (int64_t)t * B.arows * B.acols + (int64_t)row * B.acols;
        R sr = R(0), si = R(0);
        for (int j = 0; j < B.acols; ++j) {
          const cplx<S> cc = Ct[j];
          const cplx<R> v = xp[(int64_t)(cb + j) * nsys + l];
          cadd_mul<R>(sr, si, (R)cc.re, (R)cc.im, v.re, v.im);
        }
        const cf64 dv = dvec[B.d_off + (int64_t)t * dstride + l0 + l];
        cadd_mul<R>(re, im, (R)dv.re, (R)dv.im, sr, si);
      }
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

template <typename R>
void launch_h2_apply(const Problem& p, H2Operator& h, int l0, int nsys, const cplx<R>* x, int64_t xs,
                     cplx<R>* y, int64_t ys, void* /*scratch*/, hipStream_t s) {
  const int P = h.p;
  cplx<R>* xh = (cplx<R>*)h.xhat_d;
  cplx<R>* yh = (cplx<R>*)h.yhat_d;
  const int nleaf = (int)h.leaves.size();
  const bool f32 = sizeof(R) == 4;
  const int dstride = h.nsys;
  const int M = (int)h.perm.size();
  cplx<R>* xp = (cplx<R>*)h.xp_d;
  cplx<R>* yp = (cplx<R>*)h.yp_d;
  const unsigned gblk = (unsigned)(((int64_t)M * nsys + kHB - 1) / kHB);
  const int nch = (nsys + kLC - 1) / kLC;
  hipLaunchKernelGGL((k_h2_gather<R>), dim3(gblk), dim3(kHB), 0, s, h.perm_d, M, nsys, x, xs, xp);
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
  // 2. couplings (all clusters; those without core blocks get zero)
  const int ncl = (int)h.cl.size();
  if (h.store_fp64)
    hipLaunchKernelGGL((k_h2_couple<R, double>), dim3(ncl, nch), dim3(kHB), 0, s, h.core_rowptr_d, h.core_list_d,
                       h.blocks_d, h.ranks_d, (const cf64*)h.cstore_d, h.dvec_d, dstride, l0, P, nsys, xh, yh);
  else
    hipLaunchKernelGGL((k_h2_couple<R, float>), dim3(ncl, nch), dim3(kHB), 0, s, h.core_rowptr_d, h.core_list_d,
                       h.blocks_d, h.ranks_d, (const cf32*)h.cstore_d, h.dvec_d, dstride, l0, P, nsys, xh, yh);
  CQM_HIP(hipGetLastError());
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
  // 4. leaves
  const int* lvs = h.level_cl_d + h.level_off[h.nlevels];
  if (h.store_fp64) {
    if (f32)
      hipLaunchKernelGGL((k_h2_leaf_out<R, double, float>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs, h.perm_d, h.U32_d,
                         h.uleaf_off_d, P, nsys, yh, h.task_rowptr_d, h.tasks_d, h.blocks_d, h.ranks_d,
                         (const cf64*)h.cstore_d, h.dvec_d, dstride, l0, xp, yp);
    else
      hipLaunchKernelGGL((k_h2_leaf_out<R, double, double>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs, h.perm_d, h.U_d,
                         h.uleaf_off_d, P, nsys, yh, h.task_rowptr_d, h.tasks_d, h.blocks_d, h.ranks_d,
                         (const cf64*)h.cstore_d, h.dvec_d, dstride, l0, xp, yp);
  } else {
    if (f32)
      hipLaunchKernelGGL((k_h2_leaf_out<R, float, float>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs, h.perm_d, h.U32_d,
                         h.uleaf_off_d, P, nsys, yh, h.task_rowptr_d, h.tasks_d, h.blocks_d, h.ranks_d,
                         (const cf32*)h.cstore_d, h.dvec_d, dstride, l0, xp, yp);
    else
      hipLaunchKernelGGL((k_h2_leaf_out<R, float, double>), dim3(nleaf, nch), dim3(kHB), 0, s, h.cl_d, lvs, h.perm_d, h.U_d,
                         h.uleaf_off_d, P, nsys, yh, h.task_rowptr_d, h.tasks_d, h.blocks_d, h.ranks_d,
                         (const cf32*)h.cstore_d, h.dvec_d, dstride, l0, xp, yp);
  }
  CQM_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_h2_scatter<R>), dim3(gblk), dim3(kHB), 0, s, h.perm_d, M, nsys, yp, y, ys);
  CQM_HIP(hipGetLastError());
}

template void launch_h2_apply<float>(const Problem&, H2Operator&, int, int, const cf32*, int64_t, cf32*,
                                     int64_t, void*, hipStream_t);
template void launch_h2_apply<double>(const Problem&, H2Operator&, int, int, const cf64*, int64_t, cf64*,
                                      int64_t, void*, hipStream_t);

}  // namespace cqm
