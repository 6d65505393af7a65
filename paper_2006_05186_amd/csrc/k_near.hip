// Near field: pairs of triangles that share a vertex (including i = j).
//   V_ij(s) = S_ij + D_ij(s)
// S_ij: integral of 1/(4 pi |x-y|) over the pair by Duffy-type rules (one per
//       sharing pattern), computed once per mesh in FP64;
// D_ij(s) = sum_ab W_ia W_jb (exp(-s r) - 1)/(4 pi r): the bounded remainder by
//       the 6-point rule, with its r = 0 value -s/(4 pi), per frequency, FP64.
// These entries are the largest of every row and the time-domain solution
// amplifies their rounding by up to rho^-N (1e8), so this file is compiled
// without contraction into fused multiply-adds (each product and sum rounded
// on its own) and exp(-s r) - 1 is formed without cancellation.
#include "device_util.h"
#include "fp64_math.h"

namespace cqm {

namespace {
constexpr double kInv4Pi = 0.07957747154594767;  // 1/(4 pi)
constexpr double kPi = 3.141592653589793;

struct d3 {
  double x, y, z;
};
__device__ __forceinline__ d3 ld(const double* v, int k) { return d3{v[3 * k], v[3 * k + 1], v[3 * k + 2]}; }
__device__ __forceinline__ d3 sub(d3 a, d3 b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 axpy(double t, d3 a, d3 b) { return d3{b.x + t * a.x, b.y + t * a.y, b.z + t * a.z}; }
__device__ __forceinline__ double nrm(d3 a) { return sqrt(a.x * a.x + a.y * a.y + a.z * a.z); }
__device__ __forceinline__ double tri_area(d3 a, d3 b) {
  const double cx = a.y * b.z - a.z * b.y, cy = a.z * b.x - a.x * b.z, cz = a.x * b.y - a.y * b.x;
  return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
}

// Self pair: in difference coordinates the six sectors of the hexagon
// T - T carry a radial Jacobian that cancels 1/r; the radial factor (1-rho)^2
// and the inner point integral are exact, leaving one Gauss dimension along
// each hexagon edge.  Opposite edges coincide: three segments, counted twice.
__device__ double static_self(d3 A, d3 B, d3 C, const double* gx, const double* gw, int q) {
  const d3 ab = sub(B, A), ac = sub(C, A), bc = sub(C, B);
  const d3 sa[3] = {ab, ac, bc};
  const d3 sb[3] = {ac, bc, d3{-ab.x, -ab.y, -ab.z}};
  double acc = 0.0;
  for (int k = 0; k < 3; ++k) {
    const d3 dir = sub(sb[k], sa[k]);
    for (int t = 0; t < q; ++t) acc += gw[t] / nrm(axpy(gx[t], dir, sa[k]));
  }
  const double ar = tri_area(ab, ac);
  return ar * ar / (3.0 * kPi) * acc;
}

// Edge-sharing pair tau = (A,B,C), t = (A,B,D): x - y = delta e + alpha c - beta d
// depends on three coordinates; the free coordinate along the edge integrates
// to 1 - h(delta,alpha,beta) with the gauge h = max(0,delta) + max(alpha, beta - delta).
// Radial coordinates on {h = 1} reduce the integral to four planar unit-square
// pieces with Jacobians 1, p, p, 1.
__device__ double static_edge(d3 A, d3 B, d3 C, d3 D, const double* gx, const double* gw, int q) {
  const d3 e = sub(B, A), c = sub(C, A), d = sub(D, A);
  double acc = 0.0;
  for (int i = 0; i < q; ++i) {
    const double p = gx[i];
    for (int k = 0; k < q; ++k) {
      const double r = gx[k], w = gw[i] * gw[k];
      // (delta, alpha, beta, jacobian) of the four pieces
      const double pc[4][4] = {{1.0 - p, p, r, 1.0},
                               {p * (1.0 - r), p * r, 1.0, p},
                               {-p * (1.0 - r), 1.0, p * r, p},
                               {-p, r, 1.0 - p, 1.0}};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const d3 v{pc[s][0] * e.x + pc[s][1] * c.x - pc[s][2] * d.x,
                   pc[s][0] * e.y + pc[s][1] * c.y - pc[s][2] * d.y,
                   pc[s][0] * e.z + pc[s][1] * c.z - pc[s][2] * d.z};
        acc += w * pc[s][3] / nrm(v);
      }
    }
  }
  return tri_area(e, c) * tri_area(e, d) / (6.0 * kPi) * acc;
}

// Vertex-sharing pair tau = (P,A1,A2), t = (P,B1,B2): polar-type coordinates
// from P on both triangles, split where the two radial coordinates cross; the
// common radial factor integrates exactly (xi^2 -> 1/3).
__device__ double static_vertex(d3 P, d3 A1, d3 A2, d3 B1, d3 B2, const double* gx,
                                const double* gw, int q) {
  const d3 a1 = sub(A1, P), a2 = sub(A2, P), b1 = sub(B1, P), b2 = sub(B2, P);
  const d3 da = sub(a2, a1), db = sub(b2, b1);
  double acc = 0.0;
  for (int i = 0; i < q; ++i) {
    const d3 a = axpy(gx[i], da, a1);
    for (int k = 0; k < q; ++k) {
      const d3 b = axpy(gx[k], db, b1);
      const double wik = gw[i] * gw[k];
      for (int t = 0; t < q; ++t) {
        const double u = gx[t];
        const d3 v1{a.x - u * b.x, a.y - u * b.y, a.z - u * b.z};
        const d3 v2{u * a.x - b.x, u * a.y - b.y, u * a.z - b.z};
        acc += wik * gw[t] * u * (1.0 / nrm(v1) + 1.0 / nrm(v2));
      }
    }
  }
  return tri_area(a1, a2) * tri_area(b1, b2) / (3.0 * kPi) * acc;
}
}  // namespace

__global__ void k_near_static(const double* __restrict__ verts, const int32_t* __restrict__ kind,
                              const int32_t* __restrict__ vtx, int64_t nnz,
                              const double* __restrict__ gl, int q, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const int* v = vtx + 6 * k;
  const double* X = gl;
  const double* Wt = gl + q;
  double val;
  switch (kind[k]) {
    case 0:
      val = static_self(ld(verts, v[0]), ld(verts, v[1]), ld(verts, v[2]), X, Wt, q);
      break;
    case 1:
      val = static_edge(ld(verts, v[0]), ld(verts, v[1]), ld(verts, v[2]), ld(verts, v[3]), X, Wt, q);
      break;
    default:
      val = static_vertex(ld(verts, v[0]), ld(verts, v[1]), ld(verts, v[2]), ld(verts, v[3]),
                          ld(verts, v[4]), X, Wt, q);
      break;
  }
  out[k] = val;
}

void launch_near_static(const Problem& p, hipStream_t s) {
  const int64_t nnz = (int64_t)p.col.size();
  hipLaunchKernelGGL(k_near_static, dim3((nnz + 127) / 128), dim3(128), 0, s, p.dev.verts,
                     p.dev.near_kind, p.dev.near_vtx, nnz, p.dev.gl, p.opt.q_duffy,
                     p.dev.near_static);
  CQM_HIP(hipGetLastError());
}

// vals[l][k] = S_k + D_k(s_l) for near pair k (row kr[k]), system l: one
// thread per pair and frequency.  With z = -s r = x + i y and the half
// angle (sin y = 2 sh ch, cos y = 1 - 2 sh^2),
//   exp(z) - 1 = (expm1(x) (1 - 2 sh^2) - 2 sh^2) + i (1 + expm1(x)) 2 sh ch,
// free of the cancellation of exp(z) - 1 at small |s r| (library expm1 and
// sincos).
__global__ __launch_bounds__(128) void k_near_values(const double4* __restrict__ pts,
                                                     const int32_t* __restrict__ krow,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ stat,
                                                     const cf64* __restrict__ sfreq, int64_t nnz,
                                                     cf64* __restrict__ vals) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= nnz) return;
  const double sr = sfreq[l].re, si = sfreq[l].im;
  const int i = krow[k], j = col[k];
  double re = 0.0, im = 0.0;
  for (int a = 0; a < kQ; ++a) {
    const double4 tp = pts[i * kQ + a];
    for (int b = 0; b < kQ; ++b) {
      const double4 sp = pts[j * kQ + b];
      const double dx = tp.x - sp.x, dy = tp.y - sp.y, dz = tp.z - sp.z;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double ww = tp.w * sp.w;
      double fr, fi;
      if (r > 0.0) {
        const double x = -sr * r, y = -si * r;
        double sh, ch;
        sincos(0.5 * y, &sh, &ch);
        const double em1 = expm1(x), sh2 = 2.0 * sh * sh;
        fr = (em1 * (1.0 - sh2) - sh2) / r;
        fi = ((1.0 + em1) * (2.0 * sh * ch)) / r;
      } else {
        fr = -sr;
        fi = -si;
      }
      re += ww * fr;
      im += ww * fi;
    }
  }
  vals[(int64_t)l * nnz + k] = cf64{stat[k] + kInv4Pi * re, kInv4Pi * im};
}

void launch_near_values(const Problem& p, cf64* vals, hipStream_t s) {
  const int64_t nnz = (int64_t)p.col.size();
  dim3 grid((unsigned)((nnz + 127) / 128), p.Fsys);
  hipLaunchKernelGGL(k_near_values, grid, dim3(128), 0, s, p.dev.pts64, p.dev.near_row,
                     p.dev.near_col, p.dev.near_static, p.dev.s, nnz, vals);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
