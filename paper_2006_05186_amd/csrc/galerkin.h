// Galerkin entries of V(s) for one pair of triangles (FP64), used wherever
// entries are needed on demand (MACA slices and fibres of near blocks).
#pragma once
#include "device_util.h"
#include "fp64_math.h"

namespace cqm {

constexpr double kInv4PiD = 0.07957747154594767;

__device__ __forceinline__ bool tri_share_vertex(int4 a, int4 b) {
  return (a.x == b.x) | (a.x == b.y) | (a.x == b.z) | (a.y == b.x) | (a.y == b.y) |
         (a.y == b.z) | (a.z == b.x) | (a.z == b.y) | (a.z == b.z);
}

// Pair sharing no vertex: sum_ab W_ia W_jb exp(-s r)/(4 pi r), 6-point rule.
__device__ inline cf64 far_pair_entry(const double4* __restrict__ pts, int i, int j, double sr,
                                      double si) {
  double re = 0.0, im = 0.0;
  for (int a = 0; a < kQ; ++a) {
    const double4 t = pts[i * kQ + a];
    for (int b = 0; b < kQ; ++b) {
      const double4 q = pts[j * kQ + b];
      const double dx = t.x - q.x, dy = t.y - q.y, dz = t.z - q.z;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      double sn, cs;
      sincos_bounded(si * r, &sn, &cs);
      const double e = exp_nonpos(-sr * r) * t.w * q.w / r;
      re += e * cs;
      im -= e * sn;
    }
  }
  return cf64{re * kInv4PiD, im * kInv4PiD};
}

// Bounded remainder of a vertex-sharing pair: sum_ab W_ia W_jb
// (exp(-s r) - 1)/(4 pi r), with the value -s/(4 pi) at r = 0.
__device__ inline cf64 near_dynamic_entry(const double4* __restrict__ pts, int i, int j,
                                          double sr, double si) {
  double re = 0.0, im = 0.0;
  for (int a = 0; a < kQ; ++a) {
    const double4 t = pts[i * kQ + a];
    for (int b = 0; b < kQ; ++b) {
      const double4 q = pts[j * kQ + b];
      const double dx = t.x - q.x, dy = t.y - q.y, dz = t.z - q.z;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double ww = t.w * q.w;
      double fr, fi;
      if (r > 0.0) {
        const double x = -sr * r, y = -si * r;
        // from the half angle: sin y = 2 sh ch, cos y - 1 = -2 sh^2, and
        // exp(x) = 1 + expm1(x): two library calls per point pair
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
  return cf64{re * kInv4PiD, im * kInv4PiD};
}

}  // namespace cqm
