// Multivariate adaptive cross approximation of every block tensor
// (Section 5.1, Algorithm 2, inside Algorithm 3): far blocks approximate the
// coupling tensor S_b[mu,nu,k] = g(xi_r,mu, xi_c,nu, s_k) (p x p x F), near
// blocks the Galerkin block V[r,c,k].  Entries are computed on demand; the
// approximant is sum_l C_l (x)_3 d_l.
//
// One workgroup per block.  Pivoting: the first slice is frequency 0 (the
// real one), the spatial pivot is the largest residual entry of the slice
// (lowest linear index on ties), the next frequency the largest |d_l[k]| over
// frequencies not used yet.  Stop when ||C_l||_F ||d_l||_2 <= eps ||G^(l)||_F,
// with ||G^(l)||_F from the Gram identity; the last update is kept.
#include "h2_internal.h"
#include "galerkin.h"

namespace cqm {

namespace {
constexpr int kMB = 256;       // threads per block tensor
constexpr int kGC = 8;         // Gram products per pass
constexpr int kMaxSys = 1024;  // frequency systems supported by the pivot mask

struct MacaArgs {
  const BlockDesc* blocks;
  int b0;
  const double* nodes;
  int m, P;
  const int* cl;  // per cluster: begin, end, parent, leaf_id
  const int* perm;
  const double4* pts;
  const int4* vid;
  const int32_t* rowptr;
  const int32_t* col;
  const double* stat;
  const cf64* s;
  int nsys, Rcap;
  double eps;
  cf64* stage;
  cf64* dvec;
  int* ranks;
};

__device__ cf64 block_entry(const MacaArgs& A, const BlockDesc& B, int e, int k) {
  const double sr = A.s[k].re, si = A.s[k].im;
  if (B.kind != kNear) {
    const int mu = e / B.cols, nu = e % B.cols;
    const int m = A.m;
    const double* nr = A.nodes + (size_t)B.r * 3 * m;
    const double* nc = A.nodes + (size_t)B.c * 3 * m;
    const int m0 = mu / (m * m), m1 = (mu / m) % m, m2 = mu % m;
    const int n0 = nu / (m * m), n1 = (nu / m) % m, n2 = nu % m;
    const double dx = nr[m0] - nc[n0], dy = nr[m + m1] - nc[m + n1], dz = nr[2 * m + m2] - nc[2 * m + n2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double sn, cs;
    sincos_bounded(si * r, &sn, &cs);
    const double ex = exp_nonpos(-sr * r) * kInv4PiD / r;
    return cf64{ex * cs, -ex * sn};
  }
  const int i = e / B.cols, j = e % B.cols;
  const int ui = A.perm[A.cl[4 * B.r] + i], uj = A.perm[A.cl[4 * B.c] + j];
  if (tri_share_vertex(A.vid[ui], A.vid[uj])) {
    double st = 0.0;
    for (int q = A.rowptr[ui]; q < A.rowptr[ui + 1]; ++q)
      if (A.col[q] == uj) st = A.stat[q];
    const cf64 d = near_dynamic_entry(A.pts, ui, uj, sr, si);
    return cf64{st + d.re, d.im};
  }
  return far_pair_entry(A.pts, ui, uj, sr, si);
}

__device__ __forceinline__ cf64 cmul(cf64 a, cf64 b) {
  return cf64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
}  // namespace

__global__ __launch_bounds__(kMB) void k_maca(MacaArgs A) {
  const int b = A.b0 + blockIdx.x;
  const BlockDesc B = A.blocks[b];
  const int mn = B.rows * B.cols, F = A.nsys, R = A.Rcap;
  cf64* C = A.stage + B.stage_off;
  cf64* d = A.dvec + B.d_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kMB / 64;
  __shared__ double redv[NW * 2 * kGC * 2];
  __shared__ double redm[NW];
  __shared__ int redi[NW];
  __shared__ unsigned char used[kMaxSys];
  for (int k = tid; k < F; k += kMB) used[k] = 0;
  int kpiv = 0, rank = R;
  double G2 = 0.0;
  __syncthreads();
  for (int l = 0; l < R; ++l) {
    // residual slice at frequency kpiv
    double best = -1.0, nrm = 0.0;
    int bidx = 0x7fffffff;
    for (int e = tid; e < mn; e += kMB) {
      cf64 v = block_entry(A, B, e, kpiv);
      for (int t = 0; t < l; ++t) {
        const cf64 u = cmul(C[(int64_t)t * mn + e], d[(int64_t)t * F + kpiv]);
        v.re -= u.re;
        v.im -= u.im;
      }
      C[(int64_t)l * mn + e] = v;
      const double a = v.re * v.re + v.im * v.im;
      nrm += a;
      if (a > best) best = a, bidx = e;  // e increases per thread: ties keep the lower
    }
    // argmax over the workgroup (value, then lowest index)
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bidx, off, 64);
      if (ob > best || (ob == best && oi < bidx)) best = ob, bidx = oi;
    }
    nrm = wave_sum(nrm);
    __syncthreads();
    if (lane == 0) {
      redm[wv] = best;
      redi[wv] = bidx;
      redv[wv] = nrm;
    }
    __syncthreads();
    best = redm[0];
    bidx = redi[0];
    nrm = 0.0;
    for (int q = 0; q < NW; ++q) {
      if (redm[q] > best || (redm[q] == best && redi[q] < bidx)) best = redm[q], bidx = redi[q];
      nrm += redv[q];
    }
    if (!(best > 0.0)) {  // exactly zero residual slice: the approximation is exact
      rank = l;
      break;
    }
    const cf64 piv = C[(int64_t)l * mn + bidx];
    const double pn = piv.re * piv.re + piv.im * piv.im;
    // fibre through the pivot, scaled by the pivot
    for (int k = tid; k < F; k += kMB) {
      cf64 v = block_entry(A, B, bidx, k);
      for (int t = 0; t < l; ++t) {
        const cf64 u = cmul(C[(int64_t)t * mn + bidx], d[(int64_t)t * F + k]);
        v.re -= u.re;
        v.im -= u.im;
      }
      d[(int64_t)l * F + k] = cf64{(v.re * piv.re + v.im * piv.im) / pn, (v.im * piv.re - v.re * piv.im) / pn};
    }
    __syncthreads();
    // Gram identity: ||G^(l)||^2 = ||G^(l-1)||^2 + ||C_l||^2 ||d_l||^2
    //                             + 2 Re sum_t <C_l, C_t> <d_l, d_t>
    double dn = 0.0;
    for (int k = tid; k < F; k += kMB) {
      const cf64 v = d[(int64_t)l * F + k];
      dn += v.re * v.re + v.im * v.im;
    }
    dn = block_sum(dn, redv);
    double cross = 0.0;
    for (int t0 = 0; t0 < l; t0 += kGC) {
      double a[2 * kGC], bb[2 * kGC];
#pragma unroll
      for (int u = 0; u < 2 * kGC; ++u) a[u] = bb[u] = 0.0;
      for (int e = tid; e < mn; e += kMB) {
        const cf64 x = C[(int64_t)l * mn + e];
#pragma unroll
        for (int u = 0; u < kGC; ++u)
          if (t0 + u < l) {
            const cf64 y = C[(int64_t)(t0 + u) * mn + e];
            a[2 * u] += x.re * y.re + x.im * y.im;
            a[2 * u + 1] += x.im * y.re - x.re * y.im;
          }
      }
      for (int k = tid; k < F; k += kMB) {
        const cf64 x = d[(int64_t)l * F + k];
#pragma unroll
        for (int u = 0; u < kGC; ++u)
          if (t0 + u < l) {
            const cf64 y = d[(int64_t)(t0 + u) * F + k];
            bb[2 * u] += x.re * y.re + x.im * y.im;
            bb[2 * u + 1] += x.im * y.re - x.re * y.im;
          }
      }
#pragma unroll
      for (int u = 0; u < 2 * kGC; ++u) {
        a[u] = wave_sum(a[u]);
        bb[u] = wave_sum(bb[u]);
      }
      __syncthreads();
      if (lane == 0)
        for (int u = 0; u < 2 * kGC; ++u) {
          redv[(wv * 2 * kGC + u) * 2] = a[u];
          redv[(wv * 2 * kGC + u) * 2 + 1] = bb[u];
        }
      __syncthreads();
      for (int u = 0; u < kGC && t0 + u < l; ++u) {
        double cr = 0, ci = 0, dr = 0, di = 0;
        for (int q = 0; q < NW; ++q) {
          cr += redv[(q * 2 * kGC + 2 * u) * 2];
          ci += redv[(q * 2 * kGC + 2 * u + 1) * 2];
          dr += redv[(q * 2 * kGC + 2 * u) * 2 + 1];
          di += redv[(q * 2 * kGC + 2 * u + 1) * 2 + 1];
        }
        cross += cr * dr - ci * di;  // Re(<C_l,C_t><d_l,d_t>)
      }
    }
    G2 += nrm * dn + 2.0 * cross;
    if (tid == 0) used[kpiv] = 1;
    if (sqrt(nrm * dn) <= A.eps * sqrt(fmax(G2, 0.0))) {
      rank = l + 1;
      break;
    }
    __syncthreads();
    // next frequency pivot: largest |d_l[k]| among unused frequencies
    double bv = -1.0;
    int bk = 0x7fffffff;
    for (int k = tid; k < F; k += kMB)
      if (!used[k]) {
        const cf64 v = d[(int64_t)l * F + k];
        const double a = v.re * v.re + v.im * v.im;
        if (a > bv) bv = a, bk = k;
      }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bk, off, 64);
      if (ob > bv || (ob == bv && oi < bk)) bv = ob, bk = oi;
    }
    __syncthreads();
    if (lane == 0) {
      redm[wv] = bv;
      redi[wv] = bk;
    }
    __syncthreads();
    bv = redm[0];
    bk = redi[0];
    for (int q = 1; q < NW; ++q)
      if (redm[q] > bv || (redm[q] == bv && redi[q] < bk)) bv = redm[q], bk = redi[q];
    if (bk == 0x7fffffff) {  // every frequency used: the tensor is reproduced
      rank = l + 1;
      break;
    }
    kpiv = bk;
    __syncthreads();
  }
  if (tid == 0) A.ranks[b] = rank;
}

void launch_maca(const Problem& p, H2Operator& h, int b0, int nb, hipStream_t s) {
  require(p.Fsys <= kMaxSys, CQM_EINVAL, "too many frequency systems for MACA");
  MacaArgs A;
  A.blocks = h.blocks_d;
  A.b0 = b0;
  A.nodes = h.nodes_d;
  A.m = h.m;
  A.P = h.p;
  A.cl = h.cl_d;
  A.perm = h.perm_d;
  A.pts = p.dev.pts64;
  A.vid = p.dev.vid;
  A.rowptr = p.dev.near_rowptr;
  A.col = p.dev.near_col;
  A.stat = p.dev.near_static;
  A.s = p.dev.s;
  A.nsys = p.Fsys;
  A.Rcap = h.Rcap;
  A.eps = p.opt.eps_aca;
  A.stage = h.stage_d;
  A.dvec = h.dvec_d;
  A.ranks = h.ranks_d;
  hipLaunchKernelGGL(k_maca, dim3(nb), dim3(kMB), 0, s, A);
  CQM_HIP(hipGetLastError());
}

// Apply-ready slices: cores and near blocks are copied (converted to the
// storage precision); small far blocks are expanded to U_r C_t U_c^T.
template <typename S>
__global__ __launch_bounds__(256) void k_maca_finalize(const BlockDesc* __restrict__ blocks, int b0,
                                                       const int* __restrict__ ranks,
                                                       const cf64* __restrict__ stage,
                                                       const double* __restrict__ Ufull,
                                                       const int64_t* __restrict__ uoff, int P,
                                                       cplx<S>* __restrict__ out) {
  const int b = b0 + blockIdx.x;
  const int t = blockIdx.y;
  if (t >= ranks[b]) return;
  const BlockDesc B = blocks[b];
  const cf64* Ct = stage + B.stage_off + (int64_t)t * B.rows * B.cols;
  cplx<S>* O = out + B.c_off + (int64_t)t * B.arows * B.acols;
  if (B.kind != kFarExpanded) {
    for (int e = threadIdx.x; e < B.rows * B.cols; e += blockDim.x) {
      cplx<S> v;
      v.re = (S)Ct[e].re;
      v.im = (S)Ct[e].im;
      O[e] = v;
    }
    return;
  }
  // expanded far block: O = U_r C_t U_c^T, kTsh / P rows of T = U_r C_t at
  // a time (16 rows for p <= 64, 2 for p = 512)
  constexpr int kTsh = 1024;
  __shared__ cf64 Tsh[kTsh];
  const int rows_per = max(1, kTsh / P);
  const double* Ur = Ufull + uoff[B.r];
  const double* Uc = Ufull + uoff[B.c];
  for (int i0 = 0; i0 < B.arows; i0 += rows_per) {
    const int nr = min(rows_per, B.arows - i0);
    for (int e = threadIdx.x; e < nr * P; e += blockDim.x) {
      const int i = i0 + e / P, nu = e % P;
      double re = 0.0, im = 0.0;
      for (int mu = 0; mu < P; ++mu) {
        const double u = Ur[(int64_t)i * P + mu];
        const cf64 c = Ct[(int64_t)mu * P + nu];
        re += u * c.re;
        im += u * c.im;
      }
      Tsh[e] = cf64{re, im};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nr * B.acols; e += blockDim.x) {
      const int ii = e / B.acols, j = e % B.acols;
      double re = 0.0, im = 0.0;
      for (int nu = 0; nu < P; ++nu) {
        const double u = Uc[(int64_t)j * P + nu];
        re += Tsh[ii * P + nu].re * u;
        im += Tsh[ii * P + nu].im * u;
      }
      cplx<S> v;
      v.re = (S)re;
      v.im = (S)im;
      O[(int64_t)(i0 + ii) * B.acols + j] = v;
    }
    __syncthreads();
  }
}

void launch_maca_finalize_batch(const Problem& p, H2Operator& h, int b0, int nb, hipStream_t s) {
  require(h.p <= 1024, CQM_EINVAL, "interpolation rank above 1024 is not supported");
  const size_t lds = 0;
  dim3 grid(nb, h.Rcap);
  if (h.store_fp64)
    hipLaunchKernelGGL((k_maca_finalize<double>), grid, dim3(256), lds, s, h.blocks_d, b0, h.ranks_d,
                       h.stage_d, h.Ufull_d, h.ufull_off_d, h.p, (cf64*)h.cstore_d);
  else
    hipLaunchKernelGGL((k_maca_finalize<float>), grid, dim3(256), lds, s, h.blocks_d, b0, h.ranks_d,
                       h.stage_d, h.Ufull_d, h.ufull_off_d, h.p, (cf32*)h.cstore_d);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
