// Hypersingular operator D(s) (Section 2.2, eq. wavebio) on the continuous
// piecewise-linear space S_h^1 (Section 3.2): Galerkin matrix
// D_l[p, j] = <phi_p, D(s_l) phi_j> over the hat functions of the mesh
// vertices, formed by integration by parts on the closed surface,
//   int int G(x - y, s) [curl phi_j(y) . curl phi_p(x) + s^2 n_x.n_y phi_j(y) phi_p(x)],
// G = exp(-s r)/(4 pi r), the sign with which D is elliptic (Section 3.1).
// On a flat triangle the barycentric coordinate of vertex a has the constant
// surface curl -e_a/(2|tau|), e_a = P_{a+2} - P_{a+1}; so the first term
// is a piecewise-constant single layer applied to the vector density
// u = sum_b x_b e_b / (2|t|), and the second a single layer with linear
// weights on both triangles.
//
// Quadrature (the single layer's pair classes): pairs sharing no vertex by
// the 6-point rule on both triangles, matrix-free; pairs sharing a vertex by
// the static part 1/(4 pi r) -- weighted by lambda_a(x) lambda_b(y) through
// the Sauter-Schwab transformations of the unit 4-cube (identical triangles,
// common edge, common vertex; q Gauss points per axis), once per mesh -- and
// the bounded remainder (exp(-s r) - 1)/(4 pi r) by the 6-point rule per
// frequency; the piecewise-constant entries of the curl term reuse the
// single layer's static near values.  FP64 throughout, no contraction into
// fused multiply-adds (as the other near-field kernels).
//
// Apply, per frequency: (1) per source triangle the curl density and the
// weighted point values of the linear function; (2) far pairs, split over the
// sources, into per-(triangle, local vertex) partial sums; (3) per target
// triangle the near pairs plus the partial sums in a fixed order; (4) per
// vertex the sum over its incident (triangle, local vertex) slots.
#include <algorithm>

#include "device_util.h"
#include "fp64_math.h"

namespace cqm {

namespace {
constexpr double kInv4Pi = 0.07957747154594767;
constexpr int kHsTgt = 128; // target triangles (threads) per workgroup
constexpr int kHsTs = 16;   // source triangles per LDS tile
constexpr int kHsFT = 3;    // frequencies per workgroup
constexpr int kHsWaves = 4096;

struct w3 {
  double x, y, z;
};
__device__ __forceinline__ w3 vat(const double* v, int k) { return w3{v[3 * k], v[3 * k + 1], v[3 * k + 2]}; }
__device__ __forceinline__ w3 sub(w3 a, w3 b) { return w3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot3(w3 a, w3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ double twice_area(w3 a, w3 b) {
  const double cx = a.y * b.z - a.z * b.y, cy = a.z * b.x - a.x * b.z, cz = a.x * b.y - a.y * b.x;
  return sqrt(cx * cx + cy * cy + cz * cz);
}
// e_a = P_{a+2} - P_{a+1} of the triangle with vertex ids v
__device__ __forceinline__ void edges(const double* verts, int4 v, w3 e[3]) {
  const w3 P0 = vat(verts, v.x), P1 = vat(verts, v.y), P2 = vat(verts, v.z);
  e[0] = sub(P2, P1);
  e[1] = sub(P0, P2);
  e[2] = sub(P1, P0);
}

// One Sauter-Schwab node: x = X0 + x1 (X1 - X0) + x2 (X2 - X1) on the target
// triangle, y likewise on the source; adds jw / |x - y| times the products
// of the barycentric weights (1 - x1, x1 - x2, x2) x (1 - y1, y1 - y2, y2).
__device__ __forceinline__ void ss_node(const w3* X, const w3* Y, double x1, double x2, double y1,
                                        double y2, double jw, double acc[3][3]) {
  const double bx[3] = {1.0 - x1, x1 - x2, x2}, by[3] = {1.0 - y1, y1 - y2, y2};
  const double dx = bx[0] * X[0].x + bx[1] * X[1].x + bx[2] * X[2].x -
                    (by[0] * Y[0].x + by[1] * Y[1].x + by[2] * Y[2].x);
  const double dy = bx[0] * X[0].y + bx[1] * X[1].y + bx[2] * X[2].y -
                    (by[0] * Y[0].y + by[1] * Y[1].y + by[2] * Y[2].y);
  const double dz = bx[0] * X[0].z + bx[1] * X[1].z + bx[2] * X[2].z -
                    (by[0] * Y[0].z + by[1] * Y[1].z + by[2] * Y[2].z);
  const double f = jw / sqrt(dx * dx + dy * dy + dz * dz);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] += f * bx[a] * by[b];
}
}  // namespace

// Static weighted integrals of every near pair, stored [k][a][b] in the
// local vertex orders of the row and column triangles.  Vertex lists per
// class as the near-field planner gives them: identical (A B C), edge
// (A B C D: shared edge A B, C in the row triangle, D in the column one),
// vertex (P A1 A2 B1 B2).
__global__ void k_nearD_static(const double* __restrict__ verts, const int32_t* __restrict__ kind,
                               const int32_t* __restrict__ vtx, const int32_t* __restrict__ krow,
                               const int32_t* __restrict__ col, const int4* __restrict__ vid,
                               int64_t nnz, const double* __restrict__ gl, int q,
                               double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int* v = vtx + 6 * k;
  const int kd = kind[k];
  int gx[3] = {v[0], v[1], v[2]}, gy[3];
  if (kd == 0) {
    gy[0] = v[0], gy[1] = v[1], gy[2] = v[2];
  } else if (kd == 1) {
    gy[0] = v[0], gy[1] = v[1], gy[2] = v[3];
  } else {
    gy[0] = v[0], gy[1] = v[3], gy[2] = v[4];
  }
  w3 X[3], Y[3];
  for (int a = 0; a < 3; ++a) {
    X[a] = vat(verts, gx[a]);
    Y[a] = vat(verts, gy[a]);
  }
  const double* t = gl;
  const double* w = gl + q;
  double acc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i0 = 0; i0 < q; ++i0) {
    const double xi = t[i0];
    for (int i1 = 0; i1 < q; ++i1) {
      const double e1 = t[i1];
      for (int i2 = 0; i2 < q; ++i2) {
        const double e2 = t[i2];
        for (int i3 = 0; i3 < q; ++i3) {
          const double e3 = t[i3];
          const double wt = w[i0] * w[i1] * w[i2] * w[i3];
          if (kd == 0) {
            const double j = wt * xi * xi * xi * e1 * e1 * e2;
            ss_node(X, Y, xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1), j, acc);
            ss_node(X, Y, xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2), j, acc);
            ss_node(X, Y, xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2), j, acc);
            ss_node(X, Y, xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3), j, acc);
            ss_node(X, Y, xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2), j, acc);
            ss_node(X, Y, xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), j, acc);
          } else if (kd == 1) {
            const double j1 = wt * xi * xi * xi * e1 * e1, j2 = j1 * e2;
            ss_node(X, Y, xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2), j1, acc);
            ss_node(X, Y, xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), j2, acc);
            ss_node(X, Y, xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3, j2, acc);
            ss_node(X, Y, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1, j2, acc);
            ss_node(X, Y, xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2, j2, acc);
          } else {
            const double j = wt * xi * xi * xi * e2;
            ss_node(X, Y, xi, xi * e1, xi * e2, xi * e2 * e3, j, acc);
            ss_node(X, Y, xi * e2, xi * e2 * e3, xi, xi * e1, j, acc);
          }
        }
      }
    }
  }
  // surface elements (2|X|)(2|Y|) over the reference measure, times 1/(4 pi)
  const double scale = twice_area(sub(X[1], X[0]), sub(X[2], X[0])) *
                       twice_area(sub(Y[1], Y[0]), sub(Y[2], Y[0])) * kInv4Pi;
  const int4 ti = vid[krow[k]], tj = vid[col[k]];
  const int ri[3] = {ti.x, ti.y, ti.z}, rj[3] = {tj.x, tj.y, tj.z};
  double* o = out + 9 * k;
  for (int a = 0; a < 3; ++a) {
    int la = 0;
    for (int c = 0; c < 3; ++c)
      if (ri[c] == gx[a]) la = c;
    for (int b = 0; b < 3; ++b) {
      int lb = 0;
      for (int c = 0; c < 3; ++c)
        if (rj[c] == gy[b]) lb = c;
      o[3 * la + lb] = acc[a][b] * scale;
    }
  }
}

// src[l][j] = { u (3 complex): sum_b x_b e_b / (2|t_j|),
//               g (6 complex): W_jk sum_b lambda_b(point k) x_b }
__global__ __launch_bounds__(256) void k_hs_source(const cf64* __restrict__ x, int64_t xs,
                                                   const double* __restrict__ verts,
                                                   const int4* __restrict__ vid,
                                                   const double4* __restrict__ pts, int M,
                                                   HsRule rule, cf64* __restrict__ src) {
  const int l = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= M) return;
  const int4 v = vid[j];
  const cf64* xl = x + (int64_t)l * xs;
  const cf64 xb[3] = {xl[v.x], xl[v.y], xl[v.z]};
  w3 e[3];
  edges(verts, v, e);
  const double inv = 1.0 / twice_area(e[2], sub(vat(verts, v.z), vat(verts, v.x)));
  cf64* o = src + ((int64_t)l * M + j) * 9;
  const double ex[3] = {e[0].x, e[1].x, e[2].x}, ey[3] = {e[0].y, e[1].y, e[2].y},
               ez[3] = {e[0].z, e[1].z, e[2].z};
  const double* comp[3] = {ex, ey, ez};
  for (int d = 0; d < 3; ++d) {
    double re = 0.0, im = 0.0;
    for (int b = 0; b < 3; ++b) {
      re += comp[d][b] * xb[b].re;
      im += comp[d][b] * xb[b].im;
    }
    o[d] = cf64{re * inv, im * inv};
  }
  for (int k = 0; k < kQ; ++k) {
    const double wk = pts[j * kQ + k].w;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < 3; ++b) {
      re += rule.bary[k][b] * xb[b].re;
      im += rule.bary[k][b] * xb[b].im;
    }
    o[3 + k] = cf64{wk * re, wk * im};
  }
}

// Far pairs, matrix-free: one thread per target triangle and kHsFT
// frequencies; source triangles through LDS; the source range split over
// blockIdx.z.  Per target: A = sum_t V_tau,t u_t (curl term) and, per local
// vertex a, Z_a = sum_k W_k lambda_a(k) sum_t (n_tau.n_t) sum_l G(x_k - y_l)
// g_t,l (mass term, folded over the target points as they are visited); the
// partial result per local vertex a is c_a.A + s^2 Z_a.
__global__ __launch_bounds__(kHsTgt) void k_hs_far(const double4* __restrict__ pts,
                                                   const int4* __restrict__ vid,
                                                   const double4* __restrict__ nrm,
                                                   const double* __restrict__ verts, int M,
                                                   const cf64* __restrict__ sfreq, int l0, int nsys,
                                                   const cf64* __restrict__ src, HsRule rule,
                                                   cf64* __restrict__ partial, int chunk,
                                                   const double* __restrict__ ftab,
                                                   const double* __restrict__ eau,
                                                   const double* __restrict__ pbu) {
  const int lt = blockIdx.y * kHsFT;
  const int nl = min(kHsFT, nsys - lt);
  const int i = blockIdx.x * kHsTgt + threadIdx.x;
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
  // -Re(s) and Im(s) in the steps of the exponential and the fine
  // sine/cosine tables (staged in LDS below)
  double fe[kHsFT], fp[kHsFT];
  double Are[kHsFT][3], Aim[kHsFT][3], Zre[kHsFT][3], Zim[kHsFT][3];
#pragma unroll
  for (int l = 0; l < kHsFT; ++l) {
    fe[l] = l < nl ? eau[l0 + lt + l] : 0.0;
    fp[l] = l < nl ? pbu[l0 + lt + l] : 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) Are[l][d] = Aim[l][d] = Zre[l][d] = Zim[l][d] = 0.0;
  }
  __shared__ double4 sp[kHsTs * kQ];
  __shared__ double4 sn[kHsTs];
  __shared__ int4 sv[kHsTs];
  __shared__ cf64 sx[kHsTs * kHsFT * 9];
  __shared__ __align__(16) double stab[256 + kFp64Tab512Len];
  for (int k = threadIdx.x; k < 256 + kFp64Tab512Len; k += kHsTgt)
    stab[k] = ftab[k < 256 ? k : kFp64Tab512Off + (k - 256)];
  const int j0 = blockIdx.z * chunk;
  const int j1 = min(M, j0 + chunk);
  for (int jt = j0; jt < j1; jt += kHsTs) {
    const int nt = min(kHsTs, j1 - jt);
    __syncthreads();
    for (int k = threadIdx.x; k < nt * kQ; k += kHsTgt) sp[k] = pts[jt * kQ + k];
    for (int k = threadIdx.x; k < nt; k += kHsTgt) {
      sv[k] = vid[jt + k];
      sn[k] = nrm[jt + k];
    }
    for (int k = threadIdx.x; k < nt * kHsFT * 9; k += kHsTgt) {
      const int jj = k / (kHsFT * 9), r = k % (kHsFT * 9), l = r / 9, c = r % 9;
      sx[k] = l < nl ? src[((int64_t)(lt + l) * M + jt + jj) * 9 + c] : cf64{0.0, 0.0};
    }
    __syncthreads();
    for (int jj = 0; jj < nt; ++jj) {
      const int4 w4 = sv[jj];
      if ((tv.x == w4.x) | (tv.x == w4.y) | (tv.x == w4.z) | (tv.y == w4.x) | (tv.y == w4.y) |
          (tv.y == w4.z) | (tv.z == w4.x) | (tv.z == w4.y) | (tv.z == w4.z))
        continue;
      const double4 nj = sn[jj];
      const double nn = ni.x * nj.x + ni.y * nj.y + ni.z * nj.z;
      const cf64* xs = sx + jj * kHsFT * 9;
      double vre[kHsFT], vim[kHsFT];
#pragma unroll
      for (int l = 0; l < kHsFT; ++l) vre[l] = vim[l] = 0.0;
#pragma unroll 1
      for (int a = 0; a < kQ; ++a) {
        double hre[kHsFT], him[kHsFT], gre[kHsFT], gim[kHsFT];
#pragma unroll
        for (int l = 0; l < kHsFT; ++l) hre[l] = him[l] = gre[l] = gim[l] = 0.0;
        for (int b = 0; b < kQ; ++b) {
          const double4 q = sp[jj * kQ + b];
          const double dx = tx[a] - q.x, dy = ty[a] - q.y, dz = tz[a] - q.z;
          const double r2 = dx * dx + dy * dy + dz * dz;
          const double ir = rsqrt(r2);  // far pairs: r > 0
          const double r = r2 * ir;
#pragma unroll
          for (int l = 0; l < kHsFT; ++l) {
            double sn, c;
            sincos_tabu512(fp[l] * r, stab + 256, &sn, &c);
            const double e = ir * exp_tabu(fmax(fe[l] * r, -261474.0), stab);
            const double Gr = e * c, Gi = -e * sn;  // exp(-s r)/r
            hre[l] += Gr * q.w;
            him[l] += Gi * q.w;
            const cf64 g = xs[l * 9 + 3 + b];
            gre[l] += Gr * g.re - Gi * g.im;
            gim[l] += Gr * g.im + Gi * g.re;
          }
        }
        const double twa = tw[a];
        const double f0 = twa * nn * rule.bary[a][0], f1 = twa * nn * rule.bary[a][1],
                     f2 = twa * nn * rule.bary[a][2];
#pragma unroll
        for (int l = 0; l < kHsFT; ++l) {
          vre[l] += twa * hre[l];
          vim[l] += twa * him[l];
          Zre[l][0] += f0 * gre[l];
          Zim[l][0] += f0 * gim[l];
          Zre[l][1] += f1 * gre[l];
          Zim[l][1] += f1 * gim[l];
          Zre[l][2] += f2 * gre[l];
          Zim[l][2] += f2 * gim[l];
        }
      }
#pragma unroll
      for (int l = 0; l < kHsFT; ++l)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const cf64 u = xs[l * 9 + d];
          Are[l][d] += vre[l] * u.re - vim[l] * u.im;
          Aim[l][d] += vre[l] * u.im + vim[l] * u.re;
        }
    }
  }
  if (i < M) {
    w3 e[3];
    edges(verts, tv, e);
    const double inv = 1.0 / twice_area(e[2], sub(vat(verts, tv.z), vat(verts, tv.x)));
#pragma unroll
    for (int l = 0; l < kHsFT; ++l) {
      if (l >= nl) continue;
      const cf64 sv = sfreq[l0 + lt + l];
      const double s2r = sv.re * sv.re - sv.im * sv.im, s2i = 2.0 * sv.re * sv.im;
      cf64* o = partial + (((int64_t)blockIdx.z * nsys + lt + l) * M + i) * 3;
      for (int a = 0; a < 3; ++a) {
        const double cx = e[a].x * inv, cy = e[a].y * inv, cz = e[a].z * inv;
        double re = cx * Are[l][0] + cy * Are[l][1] + cz * Are[l][2];
        double im = cx * Aim[l][0] + cy * Aim[l][1] + cz * Aim[l][2];
        const double wr = Zre[l][a], wi = Zim[l][a];
        re += s2r * wr - s2i * wi;
        im += s2r * wi + s2i * wr;
        o[a] = cf64{re * kInv4Pi, im * kInv4Pi};
      }
    }
  }
}

// z[l][i][a] = sum_q partial[q][l][i][a] + near pairs of row i: per pair the
// single-layer value V = Vstatic + 6x6 rule of the remainder and the weighted
// values W_ab = Wstatic_ab + 6x6 rule of the weighted remainder, combined as
// sum_b ((c_a . c_b) V + s^2 (n_i . n_j) W_ab) x[vertex b of j].
__global__ __launch_bounds__(128) void k_hs_near(
    const cf64* __restrict__ partial, int S, int nsys, int M, const double4* __restrict__ pts,
    const int4* __restrict__ vid, const double4* __restrict__ nrm, const double* __restrict__ verts,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ vstat, const double* __restrict__ wstat,
    const cf64* __restrict__ sfreq, int l0, const cf64* __restrict__ x, int64_t xs, HsRule rule,
    cf64* __restrict__ z) {
  const int l = blockIdx.y;
  const int i = blockIdx.x * 128 + threadIdx.x;
  if (i >= M) return;
  double zr[3] = {0, 0, 0}, zi[3] = {0, 0, 0};
  for (int q = 0; q < S; ++q) {
    const cf64* pp = partial + (((int64_t)q * nsys + l) * M + i) * 3;
    for (int a = 0; a < 3; ++a) {
      zr[a] += pp[a].re;
      zi[a] += pp[a].im;
    }
  }
  const double sr = sfreq[l0 + l].re, si = sfreq[l0 + l].im;
  const double s2r = sr * sr - si * si, s2i = 2.0 * sr * si;
  const int4 tv = vid[i];
  const double4 ni = nrm[i];
  w3 ei[3];
  edges(verts, tv, ei);
  const double invi = 1.0 / twice_area(ei[2], sub(vat(verts, tv.z), vat(verts, tv.x)));
  const cf64* xl = x + (int64_t)l * xs;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
    const int j = col[k];
    const int4 sv = vid[j];
    const double4 nj = nrm[j];
    w3 ej[3];
    edges(verts, sv, ej);
    const double invj = 1.0 / twice_area(ej[2], sub(vat(verts, sv.z), vat(verts, sv.x)));
    double Vr = 0.0, Vi = 0.0, Wr[3][3], Wi[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Wr[a][b] = Wi[a][b] = 0.0;
    for (int a = 0; a < kQ; ++a) {
      const double4 tp = pts[i * kQ + a];
      double tr[3] = {0, 0, 0}, ti[3] = {0, 0, 0};
      double hr = 0.0, hi = 0.0;
      for (int b = 0; b < kQ; ++b) {
        const double4 sp = pts[j * kQ + b];
        const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double fr, fi;  // (exp(-s r) - 1)/r without cancellation; -s at r = 0
        if (r > 0.0) {
          double sh, ch;
          sincos(-0.5 * si * r, &sh, &ch);
          const double em1 = expm1(-sr * r), sh2 = 2.0 * sh * sh;
          fr = (em1 * (1.0 - sh2) - sh2) / r;
          fi = ((1.0 + em1) * (2.0 * sh * ch)) / r;
        } else {
          fr = -sr;
          fi = -si;
        }
        hr += sp.w * fr;
        hi += sp.w * fi;
        for (int c = 0; c < 3; ++c) {
          const double f = sp.w * rule.bary[b][c];
          tr[c] += f * fr;
          ti[c] += f * fi;
        }
      }
      Vr += tp.w * hr;
      Vi += tp.w * hi;
      for (int c = 0; c < 3; ++c) {
        const double f = tp.w * rule.bary[a][c];
        for (int b = 0; b < 3; ++b) {
          Wr[c][b] += f * tr[b];
          Wi[c][b] += f * ti[b];
        }
      }
    }
    Vr = vstat[k] + kInv4Pi * Vr;
    Vi = kInv4Pi * Vi;
    const double nn = ni.x * nj.x + ni.y * nj.y + ni.z * nj.z;
    const cf64 xb[3] = {xl[sv.x], xl[sv.y], xl[sv.z]};
    const double* ws = wstat + 9 * (int64_t)k;
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b) {
        const double cc = dot3(ei[a], ej[b]) * invi * invj;
        const double wr = ws[3 * a + b] + kInv4Pi * Wr[a][b], wi = kInv4Pi * Wi[a][b];
        // cc V + s^2 nn W
        const double er = cc * Vr + nn * (s2r * wr - s2i * wi);
        const double eim = cc * Vi + nn * (s2r * wi + s2i * wr);
        zr[a] += er * xb[b].re - eim * xb[b].im;
        zi[a] += er * xb[b].im + eim * xb[b].re;
      }
    }
  }
  cf64* o = z + ((int64_t)l * M + i) * 3;
  for (int a = 0; a < 3; ++a) o[a] = cf64{zr[a], zi[a]};
}

// y[l][p] = sum over the (triangle, local vertex) slots of vertex p, in the
// order of the vertex-to-slot table.
__global__ __launch_bounds__(256) void k_hs_gather(const cf64* __restrict__ z, int M,
                                                   const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ slot, int nv,
                                                   cf64* __restrict__ y, int64_t ys) {
  const int l = blockIdx.y;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= nv) return;
  double re = 0.0, im = 0.0;
  const cf64* zl = z + (int64_t)l * M * 3;
  for (int k = ptr[p]; k < ptr[p + 1]; ++k) {
    const cf64 v = zl[slot[k]];
    re += v.re;
    im += v.im;
  }
  y[(int64_t)l * ys + p] = cf64{re, im};
}

int hs_splits(int M, int nsys, int* chunk_out) {
  const int tiles = ((M + kHsTgt - 1) / kHsTgt) * ((nsys + kHsFT - 1) / kHsFT);
  int S = (kHsWaves + tiles - 1) / tiles;
  const int maxS = (M + kHsTs - 1) / kHsTs;
  S = std::max(1, std::min(S, maxS));
  int chunk = (M + S - 1) / S;
  chunk = ((chunk + kHsTs - 1) / kHsTs) * kHsTs;
  if (chunk_out) *chunk_out = chunk;
  return (M + chunk - 1) / chunk;
}

size_t hs_partial_bytes(int M, int Fs) {
  size_t worst = 0;
  for (int nl = 1; nl <= Fs; ++nl)
    worst = std::max(worst, (size_t)hs_splits(M, nl, nullptr) * nl * (size_t)M * 3 * sizeof(cf64));
  return worst;
}

HsRule hs_rule() {
  HsRule r;
  double w[6];
  dunavant6(r.bary, w);
  return r;
}

void launch_nearD_static(const Problem& p, hipStream_t s) {
  const int64_t nnz = (int64_t)p.col.size();
  hipLaunchKernelGGL(k_nearD_static, dim3((unsigned)((nnz + 63) / 64)), dim3(64), 0, s, p.dev.verts,
                     p.dev.near_kind, p.dev.near_vtx, p.dev.near_row, p.dev.near_col, p.dev.vid, nnz,
                     p.dev.gl, p.opt.q_duffy, p.dev.nearD_static);
  CQM_HIP(hipGetLastError());
}

void launch_apply_D(const Problem& p, int l0, int nsys, const cf64* x, int64_t xs, cf64* y,
                    int64_t ys, cf64* src, cf64* partial, cf64* z, hipStream_t s) {
  const int M = (int)p.M;
  const HsRule rule = hs_rule();
  hipLaunchKernelGGL(k_hs_source, dim3((M + 255) / 256, nsys), dim3(256), 0, s, x, xs, p.dev.verts,
                     p.dev.vid, p.dev.pts64, M, rule, src);
  CQM_HIP(hipGetLastError());
  int chunk = 0;
  const int S = hs_splits(M, nsys, &chunk);
  dim3 grid((M + kHsTgt - 1) / kHsTgt, (nsys + kHsFT - 1) / kHsFT, S);
  hipLaunchKernelGGL(k_hs_far, grid, dim3(kHsTgt), 0, s, p.dev.pts64, p.dev.vid, p.dev.nrm64,
                     p.dev.verts, M, p.dev.s, l0, nsys, src, rule, partial, chunk, p.dev.ftab,
                     p.dev.ea64u, p.dev.pb64u);
  CQM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_hs_near, dim3((M + 127) / 128, nsys), dim3(128), 0, s, partial, S, nsys, M,
                     p.dev.pts64, p.dev.vid, p.dev.nrm64, p.dev.verts, p.dev.near_rowptr,
                     p.dev.near_col, p.dev.near_static, p.dev.nearD_static, p.dev.s, l0, x, xs,
                     rule, z);
  CQM_HIP(hipGetLastError());
  const int nv = (int)p.nv;
  hipLaunchKernelGGL(k_hs_gather, dim3((nv + 255) / 256, nsys), dim3(256), 0, s, z, M,
                     p.dev.v2t_ptr, p.dev.v2t, nv, y, ys);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
