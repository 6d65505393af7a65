// Host-only planning of a problem (no HIP calls, so it also builds with a
// plain C++ compiler under the address and undefined-behaviour sanitizers):
// the Gauss-Legendre rule of the Duffy integrals, Dunavant's 6-point rule and
// the near-field adjacency of Section 3.2 (pairs of triangles that share a
// vertex, with the vertex order each singular rule expects).
#include <algorithm>
#include <cmath>
#include <set>

#include "internal.h"

namespace cqm {

// Gauss-Legendre rule on [0,1] by Newton iteration on P_q.
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w) {
  // Newton's method on P_q in extended precision (x86 long double, 64-bit
  // mantissa), nodes and weights 2/((1-t^2) P_q'(t)^2) then rounded once to
  // FP64: the Duffy rules' values are the largest entries of every row, and
  // the time-domain solution amplifies their rounding by up to rho^-N
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  using L = long double;
  const L pi_l = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < q; ++i) {
    L t = std::cos(pi_l * (i + 0.75L) / (q + 0.5L));
    for (int it = 0; it < 100; ++it) {
      L p0 = 1.0L, p1 = t;
      for (int k = 2; k <= q; ++k) {
        const L p2 = ((2.0L * k - 1.0L) * t * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const L dp = q * (t * p1 - p0) / (t * t - 1.0L);
      const L dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-19L) break;
    }
    L a0 = 1.0L, a1 = t;
    for (int k = 2; k <= q; ++k) {
      const L a2 = ((2.0L * k - 1.0L) * t * a1 - (k - 1.0L) * a0) / k;
      a0 = a1;
      a1 = a2;
    }
    const L d = q * (t * a1 - a0) / (t * t - 1.0L);
    w[i] = (double)(1.0L / ((1.0L - t * t) * d * d));  // weight on [0,1] = 2/((1-t^2)P'^2) / 2
    x[i] = (double)(0.5L * (1.0L - t));
  }
  // sort ascending
  std::vector<int> idx(q);
  for (int i = 0; i < q; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return x[a] < x[b]; });
  std::vector<double> xs(q), ws(q);
  for (int i = 0; i < q; ++i) xs[i] = x[idx[i]], ws[i] = w[idx[i]];
  x = xs;
  w = ws;
}

// Dunavant's 6-point rule of degree 4 (barycentric points, weights sum to 1).
void dunavant6(double bary[6][3], double w[6]) {
  const double a = 0.445948490915965, b = 0.091576213509771;
  const double wa = 0.223381589678011, wb = 0.109951743655322;
  const double P[6][3] = {{1 - 2 * a, a, a}, {a, 1 - 2 * a, a}, {a, a, 1 - 2 * a},
                          {1 - 2 * b, b, b}, {b, 1 - 2 * b, b}, {b, b, 1 - 2 * b}};
  for (int k = 0; k < 6; ++k) {
    for (int d = 0; d < 3; ++d) bary[k][d] = P[k][d];
    w[k] = k < 3 ? wa : wb;
  }
}

// Near field: for every triangle, the triangles sharing at least one vertex
// index (itself included), with the vertex ordering each Duffy rule expects:
// kind 0 (same triangle) A B C; kind 1 (shared edge AB) A B C D, C in row
// triangle, D in column triangle; kind 2 (shared vertex P) P A1 A2 B1 B2.
void build_near(Problem& p) {
  const int64_t M = p.M;
  std::vector<std::vector<int32_t>> by_vertex(p.nv);
  for (int64_t i = 0; i < M; ++i)
    for (int k = 0; k < 3; ++k) by_vertex[p.tris[3 * i + k]].push_back((int32_t)i);
  p.rowptr.assign(M + 1, 0);
  p.col.clear();
  p.kind.clear();
  p.nvtx.clear();
  for (int64_t i = 0; i < M; ++i) {
    std::set<int32_t> cand;
    const int32_t* ti = &p.tris[3 * i];
    for (int k = 0; k < 3; ++k) cand.insert(by_vertex[ti[k]].begin(), by_vertex[ti[k]].end());
    for (int32_t j : cand) {
      const int32_t* tj = &p.tris[3 * (int64_t)j];
      int shared[3], ns = 0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          if (ti[a] == tj[b]) shared[ns++] = ti[a];
      int32_t v[6] = {0, 0, 0, 0, 0, 0};
      int kd;
      if (j == i) {
        kd = 0;
        v[0] = ti[0], v[1] = ti[1], v[2] = ti[2];
      } else if (ns == 3) {
        throw Error(CQM_EINVAL, "duplicate triangles " + std::to_string(i) + " and " + std::to_string(j));
      } else if (ns == 2) {
        kd = 1;
        // shared edge oriented by increasing vertex index: the rule for (j,i)
        // is then the mirror image of the rule for (i,j)
        v[0] = std::min(shared[0], shared[1]), v[1] = std::max(shared[0], shared[1]);
        for (int a = 0; a < 3; ++a)
          if (ti[a] != shared[0] && ti[a] != shared[1]) v[2] = ti[a];
        for (int b = 0; b < 3; ++b)
          if (tj[b] != shared[0] && tj[b] != shared[1]) v[3] = tj[b];
      } else {
        kd = 2;
        v[0] = shared[0];
        int na = 1, nb = 3;
        for (int a = 0; a < 3; ++a)
          if (ti[a] != shared[0]) v[na++] = ti[a];
        for (int b = 0; b < 3; ++b)
          if (tj[b] != shared[0]) v[nb++] = tj[b];
      }
      p.col.push_back(j);
      p.kind.push_back(kd);
      for (int k = 0; k < 6; ++k) p.nvtx.push_back(v[k]);
    }
    p.rowptr[i + 1] = (int32_t)p.col.size();
  }
}

}  // namespace cqm
