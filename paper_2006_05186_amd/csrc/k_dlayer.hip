// Double-layer operator K(s) (Section 2.2, eq. wavebio) in the Laplace
// domain, piecewise-constant Galerkin entries
//   K_ij(s) = int_tau_i int_tau_j (1 + s r) exp(-s r) (x - y).n_j / (4 pi r^3),
// r = |x - y|, n_j the unit normal of the source triangle (its vertex order).
// Pairs sharing a vertex: the static Laplace part (x - y).n_j / (4 pi r^3)
// by Duffy rules whose radial variable integrates in closed form (zero for
// identical flat triangles), computed once per mesh, plus the bounded
// remainder (exp(-s r)(1 + s r) - 1)(x - y).n_j / (4 pi r^3) by the 6-point
// rule per frequency; other pairs by the 6-point rule on the fly.  K is
// applied once per solve, to form the right-hand side (-1/2 I + K) g_D of
// the direct formulation (eq. wavegalform with a Dirichlet boundary), in FP64.
// Compiled without contraction into fused multiply-adds, like the single
// layer's near field.
#include <algorithm>

#include "device_util.h"
#include "fp64_math.h"

namespace cqm {

namespace {
constexpr double kInv4Pi = 0.07957747154594767;
constexpr double kInv2Pi = 0.15915494309189535;
constexpr int kDlTgt = 64;  // target triangles (threads) per workgroup
constexpr int kDlTs = 32;   // source triangles per LDS tile
constexpr int kDlFT = 8;    // frequencies per workgroup
constexpr int kDlWaves = 4096;

struct v3 {
  double x, y, z;
};
__device__ __forceinline__ v3 at(const double* v, int k) { return v3{v[3 * k], v[3 * k + 1], v[3 * k + 2]}; }
__device__ __forceinline__ v3 minus(v3 a, v3 b) { return v3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double norm3(v3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ double area2(v3 a, v3 b) {  // twice the triangle area
  const double cx = a.y * b.z - a.z * b.y, cy = a.z * b.x - a.x * b.z, cz = a.x * b.y - a.y * b.x;
  return sqrt(cx * cx + cy * cy + cz * cz);
}

// Edge pair tau = (A,B,C) (target), t = (A,B,D) (source, normal n): in the
// single layer's coordinates x - y = delta e + alpha c - beta d, n is
// orthogonal to e and d, so (x - y).n = alpha (c.n); with the radial measure
// rho^2 (1 - rho) the radial integral is 1/2 and four planar pieces remain.
__device__ double dl_static_edge(v3 A, v3 B, v3 C, v3 D, v3 n, const double* gx,
                                 const double* gw, int q) {
  const v3 e = minus(B, A), c = minus(C, A), d = minus(D, A);
  double acc = 0.0;
  for (int i = 0; i < q; ++i) {
    const double p = gx[i];
    for (int k = 0; k < q; ++k) {
      const double r = gx[k], w = gw[i] * gw[k];
      const double pc[4][4] = {{1.0 - p, p, r, 1.0},
                               {p * (1.0 - r), p * r, 1.0, p},
                               {-p * (1.0 - r), 1.0, p * r, p},
                               {-p, r, 1.0 - p, 1.0}};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const v3 v{pc[s][0] * e.x + pc[s][1] * c.x - pc[s][2] * d.x,
                   pc[s][0] * e.y + pc[s][1] * c.y - pc[s][2] * d.y,
                   pc[s][0] * e.z + pc[s][1] * c.z - pc[s][2] * d.z};
        const double nv = norm3(v);
        acc += w * pc[s][3] * pc[s][1] / (nv * nv * nv);
      }
    }
  }
  // |tau||t| / (2 pi) = (2|tau|)(2|t|) / (8 pi)
  return area2(e, c) * area2(e, d) * (0.25 * kInv2Pi) * dot(c, n) * acc;
}

// Vertex pair tau = (P,A1,A2), t = (P,B1,B2): polar coordinates from P on
// both, split where the radial coordinates cross; b lies in the source
// plane, so (x - y).n is xi a.n or zeta w a.n, and the radial integral is 1/2.
__device__ double dl_static_vertex(v3 P, v3 A1, v3 A2, v3 B1, v3 B2, v3 n, const double* gx,
                                   const double* gw, int q) {
  const v3 a1 = minus(A1, P), a2 = minus(A2, P), b1 = minus(B1, P), b2 = minus(B2, P);
  const v3 da = minus(a2, a1), db = minus(b2, b1);
  double acc = 0.0;
  for (int i = 0; i < q; ++i) {
    const v3 a{a1.x + gx[i] * da.x, a1.y + gx[i] * da.y, a1.z + gx[i] * da.z};
    const double an = dot(a, n);
    for (int k = 0; k < q; ++k) {
      const v3 b{b1.x + gx[k] * db.x, b1.y + gx[k] * db.y, b1.z + gx[k] * db.z};
      const double wik = gw[i] * gw[k];
      for (int t = 0; t < q; ++t) {
        const double u = gx[t];
        const v3 v1{a.x - u * b.x, a.y - u * b.y, a.z - u * b.z};
        const v3 v2{u * a.x - b.x, u * a.y - b.y, u * a.z - b.z};
        const double n1 = norm3(v1), n2 = norm3(v2);
        acc += wik * gw[t] * an * (u / (n1 * n1 * n1) + u * u / (n2 * n2 * n2));
      }
    }
  }
  return area2(a1, a2) * area2(b1, b2) * (0.25 * kInv2Pi) * acc;
}

// exp(-z)(1 + z) - 1 for z = s r: the series -sum_{k>=2} (k-1)(-z)^k / k!
// below |z| = 0.5 (24 terms: the tail is under 1e-25 of the sum), else
// formed directly.
__device__ __forceinline__ void dl_remainder(double zr, double zi, double* fr, double* fi) {
  if (zr * zr + zi * zi < 0.25) {
    double tr = 1.0, ti = 0.0, ar = 0.0, ai = 0.0;  // t = (-z)^k / k!
    for (int k = 1; k <= 24; ++k) {
      const double nr = -(tr * zr - ti * zi) / k, ni = -(tr * zi + ti * zr) / k;
      tr = nr;
      ti = ni;
      if (k >= 2) {
        ar -= (k - 1) * tr;
        ai -= (k - 1) * ti;
      }
    }
    *fr = ar;
    *fi = ai;
  } else {
    double sn, cs;
    sincos(zi, &sn, &cs);
    const double e = exp(-zr);
    // exp(-z) = e (cos zi - i sin zi); times (1 + zr + i zi)
    const double er = e * cs, ei = -e * sn;
    *fr = er * (1.0 + zr) - ei * zi - 1.0;
    *fi = er * zi + ei * (1.0 + zr);
  }
}
}  // namespace

__global__ void k_nearK_static(const double* __restrict__ verts, const int32_t* __restrict__ kind,
                               const int32_t* __restrict__ vtx, const int32_t* __restrict__ col,
                               const double4* __restrict__ nrm, int64_t nnz,
                               const double* __restrict__ gl, int q, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int* v = vtx + 6 * k;
  const double4 nj = nrm[col[k]];
  const v3 n{nj.x, nj.y, nj.z};
  double val = 0.0;  // identical flat triangles: (x - y).n = 0
  if (kind[k] == 1)
    val = dl_static_edge(at(verts, v[0]), at(verts, v[1]), at(verts, v[2]), at(verts, v[3]), n, gl,
                         gl + q, q);
  else if (kind[k] == 2)
    val = dl_static_vertex(at(verts, v[0]), at(verts, v[1]), at(verts, v[2]), at(verts, v[3]),
                           at(verts, v[4]), n, gl, gl + q, q);
  out[k] = val;
}

// vals[l][k] = static_k + sum_ab W_ia W_jb rem(s_l r)(x - y).n_j / (4 pi r^3);
// coincident points (identical pairs) contribute 0.
__global__ __launch_bounds__(128) void k_nearK_values(const double4* __restrict__ pts,
                                                      const int32_t* __restrict__ krow,
                                                      const int32_t* __restrict__ col,
                                                      const double4* __restrict__ nrm,
                                                      const double* __restrict__ stat,
                                                      const cf64* __restrict__ sfreq, int l0,
                                                      int64_t nnz, cf64* __restrict__ vals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= nnz) return;
  const double sr = sfreq[l0 + l].re, si = sfreq[l0 + l].im;
  const int i = krow[k], j = col[k];
  const double4 nj = nrm[j];
  double re = 0.0, im = 0.0;
  for (int a = 0; a < kQ; ++a) {
    const double4 tp = pts[i * kQ + a];
    for (int b = 0; b < kQ; ++b) {
      const double4 sp = pts[j * kQ + b];
      const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (!(r > 0.0)) continue;
      double fr, fi;
      dl_remainder(sr * r, si * r, &fr, &fi);
      const double g = tp.w * sp.w * (dx * nj.x + dy * nj.y + dz * nj.z) / (r * r * r);
      re += g * fr;
      im += g * fi;
    }
  }
  vals[(int64_t)l * nnz + k] = cf64{stat[k] + kInv4Pi * re, kInv4Pi * im};
}

// Far pairs, matrix-free: one thread per target triangle and kDlFT
// frequencies; source triangles staged through LDS (points, vertex ids,
// normals, coefficients); the source range split over blockIdx.z, partial
// sums reduced in a fixed order by k_dl_reduce_near.  kAdj: the adjoint
// double layer K' (normal derivative at the target, eq. wavebio), kernel
// -(1 + s r) exp(-s r)(x - y).n_x / (4 pi r^3) with the target's normal.
template <bool kAdj>
__global__ __launch_bounds__(kDlTgt) void k_dl_far(const double4* __restrict__ pts,
                                                   const int4* __restrict__ vid,
                                                   const double4* __restrict__ nrm, int M,
                                                   const cf64* __restrict__ sfreq, int l0,
                                                   int nsys, const cf64* __restrict__ x, int64_t xs,
                                                   cf64* __restrict__ partial, int chunk,
                                                   const double* __restrict__ ftab,
                                                   const double* __restrict__ eau,
                                                   const double* __restrict__ pbu) {
  const int lt = blockIdx.y * kDlFT;
  const int nl = min(kDlFT, nsys - lt);
  const int i = blockIdx.x * kDlTgt + threadIdx.x;
  const int ic = i < M ? i : M - 1;
  double tx[kQ], ty[kQ], tz[kQ], tw[kQ];
#pragma unroll
  for (int a = 0; a < kQ; ++a) {
    const double4 q = pts[ic * kQ + a];
    tx[a] = q.x;
    ty[a] = q.y;
    tz[a] = q.z;
    tw[a] = q.w;
  }
  const int4 tv = vid[ic];
  const double4 ni = nrm[ic];
  // s_l itself (for 1 + s r) and -Re(s), Im(s) in the steps of the
  // exponential and the fine sine/cosine tables (staged in LDS below)
  double sr[kDlFT], si[kDlFT], fe[kDlFT], fp[kDlFT], are[kDlFT], aim[kDlFT];
#pragma unroll
  for (int l = 0; l < kDlFT; ++l) {
    const cf64 sv = l < nl ? sfreq[l0 + lt + l] : cf64{0.0, 0.0};
    sr[l] = sv.re;
    si[l] = sv.im;
    fe[l] = l < nl ? eau[l0 + lt + l] : 0.0;
    fp[l] = l < nl ? pbu[l0 + lt + l] : 0.0;
    are[l] = 0.0;
    aim[l] = 0.0;
  }
  __shared__ double4 sp[kDlTs * kQ];
  __shared__ double4 sn[kDlTs];
  __shared__ int4 sv[kDlTs];
  __shared__ cf64 sx[kDlTs * kDlFT];
  __shared__ __align__(16) double stab[256 + kFp64Tab512Len];
  for (int k = threadIdx.x; k < 256 + kFp64Tab512Len; k += kDlTgt)
    stab[k] = ftab[k < 256 ? k : kFp64Tab512Off + (k - 256)];
  const int j0 = blockIdx.z * chunk;
  const int j1 = min(M, j0 + chunk);
  for (int jt = j0; jt < j1; jt += kDlTs) {
    const int nt = min(kDlTs, j1 - jt);
    __syncthreads();
    for (int k = threadIdx.x; k < nt * kQ; k += kDlTgt) sp[k] = pts[jt * kQ + k];
    for (int k = threadIdx.x; k < nt; k += kDlTgt) {
      sv[k] = vid[jt + k];
      sn[k] = nrm[jt + k];
    }
    for (int l = 0; l < kDlFT; ++l)
      for (int k = threadIdx.x; k < nt; k += kDlTgt)
        sx[k * kDlFT + l] = l < nl ? x[(int64_t)(lt + l) * xs + jt + k] : cf64{0.0, 0.0};
    __syncthreads();
    for (int jj = 0; jj < nt; ++jj) {
      const int4 w4 = sv[jj];
      if ((tv.x == w4.x) | (tv.x == w4.y) | (tv.x == w4.z) | (tv.y == w4.x) | (tv.y == w4.y) |
          (tv.y == w4.z) | (tv.z == w4.x) | (tv.z == w4.y) | (tv.z == w4.z))
        continue;
      const double4 nj = kAdj ? double4{-ni.x, -ni.y, -ni.z, 0.0} : sn[jj];
      double vre[kDlFT], vim[kDlFT];
#pragma unroll
      for (int l = 0; l < kDlFT; ++l) vre[l] = vim[l] = 0.0;
      for (int b = 0; b < kQ; ++b) {
        const double4 q = sp[jj * kQ + b];
#pragma unroll 1
        for (int a = 0; a < kQ; ++a) {
          const double dx = tx[a] - q.x, dy = ty[a] - q.y, dz = tz[a] - q.z;
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double r = sqrt(r2);
          const double g = tw[a] * q.w * (dx * nj.x + dy * nj.y + dz * nj.z) / (r2 * r);
#pragma unroll
          for (int l = 0; l < kDlFT; ++l) {
            double s, c;
            sincos_tabu512(fp[l] * r, stab + 256, &s, &c);
            const double e = g * exp_tabu(fmax(fe[l] * r, -261474.0), stab);
            // (1 + s r) exp(-s r) = e-scaled ((1 + sr r) + i si r)(c - i s)
            const double a1 = 1.0 + sr[l] * r, b1 = si[l] * r;
            vre[l] += e * (a1 * c + b1 * s);
            vim[l] += e * (b1 * c - a1 * s);
          }
        }
      }
#pragma unroll
      for (int l = 0; l < kDlFT; ++l) {
        const cf64 xv = sx[jj * kDlFT + l];
        are[l] += vre[l] * xv.re - vim[l] * xv.im;
        aim[l] += vre[l] * xv.im + vim[l] * xv.re;
      }
    }
  }
  if (i < M) {
#pragma unroll
    for (int l = 0; l < kDlFT; ++l)
      if (l < nl)
        partial[((int64_t)blockIdx.z * nsys + lt + l) * M + i] =
            cf64{are[l] * kInv4Pi, aim[l] * kInv4Pi};
  }
}

// y_l[i] = alpha z_l[i] + sum_q partial[q][l][i] + sum_{k in near row i}
// Knear_l[k] x_l[col k]; z may be y itself (read before the write).  With
// tpos (the adjoint) the near value of pair (i, j) is K's value of (j, i):
// the same integral with the roles exchanged.
__global__ __launch_bounds__(256) void k_dl_reduce_near(
    const cf64* __restrict__ partial, int S, int nsys, int M, const cf64* __restrict__ x,
    int64_t xs, const cf64* z, double alpha, cf64* y, int64_t ys,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ tpos, const cf64* __restrict__ nvals, int64_t nnz) {
  const int l = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < S; ++q) {
    const cf64 v = partial[((int64_t)q * nsys + l) * M + i];
    re += v.re;
    im += v.im;
  }
  const cf64* xl = x + (int64_t)l * xs;
  const cf64* nv = nvals + (int64_t)l * nnz;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
    const cf64 a = nv[tpos ? tpos[k] : k], b = xl[col[k]];
    re += a.re * b.re - a.im * b.im;
    im += a.re * b.im + a.im * b.re;
  }
  if (z) {
    const cf64 zv = z[(int64_t)l * ys + i];
    re += alpha * zv.re;
    im += alpha * zv.im;
  }
  y[(int64_t)l * ys + i] = cf64{re, im};
}

// c_l[i] = g_l[i] / |tau_i|: the piecewise-constant coefficients of the
// Dirichlet datum from its projection integrals.
__global__ __launch_bounds__(256) void k_div_area(const cf64* __restrict__ g, int64_t gs,
                                                  const double* __restrict__ area, int M,
                                                  cf64* __restrict__ c) {
  const int l = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  const cf64 v = g[(int64_t)l * gs + i];
  const double ai = area[i];
  c[(int64_t)l * M + i] = cf64{v.re / ai, v.im / ai};
}

int dl_splits(int M, int nsys, int* chunk_out) {
  const int tiles = ((M + kDlTgt - 1) / kDlTgt) * ((nsys + kDlFT - 1) / kDlFT);
  int S = (kDlWaves + tiles - 1) / tiles;
  const int maxS = (M + kDlTs - 1) / kDlTs;
  S = std::max(1, std::min(S, maxS));
  int chunk = (M + S - 1) / S;
  chunk = ((chunk + kDlTs - 1) / kDlTs) * kDlTs;
  if (chunk_out) *chunk_out = chunk;
  return (M + chunk - 1) / chunk;
}

size_t dl_partial_bytes(int M, int Fs) {
  size_t worst = 0;
  for (int nl = 1; nl <= Fs; ++nl)
    worst = std::max(worst, (size_t)dl_splits(M, nl, nullptr) * nl * (size_t)M * sizeof(cf64));
  return worst;
}

void launch_nearK_static(const Problem& p, hipStream_t s) {
  const int64_t nnz = (int64_t)p.col.size();
  hipLaunchKernelGGL(k_nearK_static, dim3((unsigned)((nnz + 127) / 128)), dim3(128), 0, s,
                     p.dev.verts, p.dev.near_kind, p.dev.near_vtx, p.dev.near_col, p.dev.nrm64, nnz,
                     p.dev.gl, p.opt.q_duffy, p.dev.nearK_static);
  CQM_HIP(hipGetLastError());
}

void launch_nearK_values(const Problem& p, cf64* vals, hipStream_t s) {
  const int64_t nnz = (int64_t)p.col.size();
  dim3 grid((unsigned)((nnz + 127) / 128), p.Fsys);
  hipLaunchKernelGGL(k_nearK_values, grid, dim3(128), 0, s, p.dev.pts64, p.dev.near_row,
                     p.dev.near_col, p.dev.nrm64, p.dev.nearK_static, p.dev.s, 0, nnz, vals);
  CQM_HIP(hipGetLastError());
}

void launch_apply_K(const Problem& p, int l0, int nsys, const cf64* x, int64_t xs, const cf64* z,
                    double alpha, cf64* y, int64_t ys, const cf64* nvals, cf64* partial,
                    bool adjoint, hipStream_t s) {
  const int M = (int)p.M;
  int chunk = 0;
  const int S = dl_splits(M, nsys, &chunk);
  dim3 grid((M + kDlTgt - 1) / kDlTgt, (nsys + kDlFT - 1) / kDlFT, S);
  if (adjoint)
    hipLaunchKernelGGL(k_dl_far<true>, grid, dim3(kDlTgt), 0, s, p.dev.pts64, p.dev.vid, p.dev.nrm64,
                       M, p.dev.s, l0, nsys, x, xs, partial, chunk, p.dev.ftab, p.dev.ea64u,
                       p.dev.pb64u);
  else
    hipLaunchKernelGGL(k_dl_far<false>, grid, dim3(kDlTgt), 0, s, p.dev.pts64, p.dev.vid, p.dev.nrm64,
                       M, p.dev.s, l0, nsys, x, xs, partial, chunk, p.dev.ftab, p.dev.ea64u,
                       p.dev.pb64u);
  CQM_HIP(hipGetLastError());
  const int64_t nnz = (int64_t)p.col.size();
  hipLaunchKernelGGL(k_dl_reduce_near, dim3((M + 255) / 256, nsys), dim3(256), 0, s, partial, S,
                     nsys, M, x, xs, z, alpha, y, ys, p.dev.near_rowptr, p.dev.near_col,
                     adjoint ? p.dev.near_tpos : nullptr, nvals + (int64_t)l0 * nnz, nnz);
  CQM_HIP(hipGetLastError());
}

void launch_div_area(const Problem& p, int nsys, const cf64* g, int64_t gs, cf64* c, hipStream_t s) {
  const int M = (int)p.M;
  hipLaunchKernelGGL(k_div_area, dim3((M + 255) / 256, nsys), dim3(256), 0, s, g, gs, p.dev.area,
                     M, c);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
