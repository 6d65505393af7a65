// Host planner of the compressed operator: cluster tree by geometric
// bisection (Section 4.1), block cluster tree with the bounding-box
// admissibility condition (eq. qadm), tensor Chebyshev interpolation bases:
// leaf matrices and transfer matrices (Section 4.2, Algorithm 1), and the
// block lists and workspace plan used by the GPU kernels.
#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>

#include "h2_internal.h"

namespace cqm {

namespace {
double box_diam(const Cluster& c) {
  double s = 0;
  for (int d = 0; d < 3; ++d) s += (c.hi[d] - c.lo[d]) * (c.hi[d] - c.lo[d]);
  return std::sqrt(s);
}
double box_dist(const Cluster& a, const Cluster& b) {
  double s = 0;
  for (int d = 0; d < 3; ++d) {
    const double g = std::max(0.0, std::max(a.lo[d] - b.hi[d], b.lo[d] - a.hi[d]));
    s += g * g;
  }
  return std::sqrt(s);
}
// Lagrange polynomial k on the nodes x[0..m-1], evaluated at t.
double lagrange(const double* x, int m, int k, double t) {
  double v = 1.0;
  for (int j = 0; j < m; ++j)
    if (j != k) v *= (t - x[j]) / (x[k] - x[j]);
  return v;
}
}  // namespace

void h2_build_structure(Problem& p, H2Operator& h) {
  const int64_t M = p.M;
  const int nmin = p.opt.n_min, m = p.opt.cheb_m;
  h.m = m;
  h.p = m * m * m;
  h.nsys = p.Fsys;
  h.Rcap = std::min(p.Fsys, 48);
  // centroids and support boxes of the triangles
  std::vector<double> cen(3 * M), tlo(3 * M), thi(3 * M);
  for (int64_t i = 0; i < M; ++i)
    for (int d = 0; d < 3; ++d) {
      double a = p.verts[3 * p.tris[3 * i] + d], b = p.verts[3 * p.tris[3 * i + 1] + d],
             c = p.verts[3 * p.tris[3 * i + 2] + d];
      cen[3 * i + d] = (a + b + c) / 3.0;
      tlo[3 * i + d] = std::min(a, std::min(b, c));
      thi[3 * i + d] = std::max(a, std::max(b, c));
    }
  h.perm.resize(M);
  std::iota(h.perm.begin(), h.perm.end(), 0);
  h.cl.clear();
  // geometric bisection: split the support box at the midpoint of its longest
  // axis (by centroid) while #r > n_min; a one-sided split falls back to the
  // median so that no cluster has a single son
  std::function<int(int, int, int, int)> rec = [&](int b, int e, int level, int parent) -> int {
    const int id = (int)h.cl.size();
    h.cl.emplace_back();
    Cluster c;
    c.begin = b;
    c.end = e;
    c.level = level;
    c.parent = parent;
    for (int d = 0; d < 3; ++d) c.lo[d] = 1e300, c.hi[d] = -1e300;
    for (int k = b; k < e; ++k)
      for (int d = 0; d < 3; ++d) {
        c.lo[d] = std::min(c.lo[d], tlo[3 * h.perm[k] + d]);
        c.hi[d] = std::max(c.hi[d], thi[3 * h.perm[k] + d]);
      }
    h.cl[id] = c;
    if (e - b > nmin) {
      int ax = 0;
      for (int d = 1; d < 3; ++d)
        if (c.hi[d] - c.lo[d] > c.hi[ax] - c.lo[ax]) ax = d;
      const double mid = 0.5 * (c.lo[ax] + c.hi[ax]);
      auto it = std::partition(h.perm.begin() + b, h.perm.begin() + e,
                               [&](int t) { return cen[3 * t + ax] <= mid; });
      int sp = (int)(it - h.perm.begin());
      if (sp == b || sp == e) {
        std::sort(h.perm.begin() + b, h.perm.begin() + e,
                  [&](int u, int v) { return cen[3 * u + ax] < cen[3 * v + ax]; });
        sp = b + (e - b) / 2;
      }
      const int s0 = rec(b, sp, level + 1, id);
      const int s1 = rec(sp, e, level + 1, id);
      h.cl[id].son[0] = s0;
      h.cl[id].son[1] = s1;
      h.cl[id].nsons = 2;
    }
    return id;
  };
  rec(0, (int)M, 0, -1);
  h.iperm.assign(M, 0);
  for (int64_t k = 0; k < M; ++k) h.iperm[h.perm[k]] = (int)k;
  const int ncl = (int)h.cl.size();
  h.leaves.clear();
  h.nlevels = 0;
  for (int c = 0; c < ncl; ++c) {
    h.nlevels = std::max(h.nlevels, h.cl[c].level + 1);
    if (h.cl[c].nsons == 0) {
      h.cl[c].leaf_id = (int)h.leaves.size();
      h.leaves.push_back(c);
    }
  }
  std::sort(h.leaves.begin(), h.leaves.end(),
            [&](int a, int b) { return h.cl[a].begin < h.cl[b].begin; });
  for (size_t k = 0; k < h.leaves.size(); ++k) h.cl[h.leaves[k]].leaf_id = (int)k;
  h.by_level.assign(h.nlevels, {});
  for (int c = 0; c < ncl; ++c) h.by_level[h.cl[c].level].push_back(c);

  // Chebyshev nodes of the first kind in each box (a flat axis is padded)
  h.nodes.assign((size_t)ncl * 3 * m, 0.0);
  for (int c = 0; c < ncl; ++c) {
    const double dg = box_diam(h.cl[c]);
    for (int d = 0; d < 3; ++d) {
      const double ctr = 0.5 * (h.cl[c].lo[d] + h.cl[c].hi[d]);
      const double half = std::max(0.5 * (h.cl[c].hi[d] - h.cl[c].lo[d]), 0.5e-12 * dg);
      for (int k = 0; k < m; ++k)
        h.nodes[((size_t)c * 3 + d) * m + k] = ctr + half * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * m));
    }
  }
  const int P = h.p;
  double bary[6][3], w6[6];
  dunavant6(bary, w6);
  auto basis_rows = [&](int c, double* out) {  // #c x p, U_c[i][mu] = sum_a W_ia L_mu(x_ia)
    const double* nx = &h.nodes[((size_t)c * 3 + 0) * m];
    const double* ny = &h.nodes[((size_t)c * 3 + 1) * m];
    const double* nz = &h.nodes[((size_t)c * 3 + 2) * m];
    const int n = h.cl[c].size();
    for (int ii = 0; ii < n; ++ii) {
      const int t = h.perm[h.cl[c].begin + ii];
      const double* A = &p.verts[3 * p.tris[3 * t]];
      const double* B = &p.verts[3 * p.tris[3 * t + 1]];
      const double* C = &p.verts[3 * p.tris[3 * t + 2]];
      double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
      const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
      double* row = out + (size_t)ii * P;
      for (int mu = 0; mu < P; ++mu) row[mu] = 0.0;
      for (int a = 0; a < 6; ++a) {
        double x[3];
        for (int d = 0; d < 3; ++d) x[d] = bary[a][0] * A[d] + bary[a][1] * B[d] + bary[a][2] * C[d];
        double lx[8], ly[8], lz[8];
        for (int k = 0; k < m; ++k) {
          lx[k] = lagrange(nx, m, k, x[0]);
          ly[k] = lagrange(ny, m, k, x[1]);
          lz[k] = lagrange(nz, m, k, x[2]);
        }
        const double wa = w6[a] * area;
        for (int a0 = 0; a0 < m; ++a0)
          for (int a1 = 0; a1 < m; ++a1)
            for (int a2 = 0; a2 < m; ++a2) row[(a0 * m + a1) * m + a2] += wa * lx[a0] * ly[a1] * lz[a2];
      }
    }
  };
  // leaf matrices
  h.uleaf_off.assign(h.leaves.size() + 1, 0);
  for (size_t k = 0; k < h.leaves.size(); ++k)
    h.uleaf_off[k + 1] = h.uleaf_off[k] + (int64_t)h.cl[h.leaves[k]].size() * P;
  h.Uleaf.assign(h.uleaf_off.back(), 0.0);
  for (size_t k = 0; k < h.leaves.size(); ++k) basis_rows(h.leaves[k], &h.Uleaf[h.uleaf_off[k]]);
  // transfer matrices E_c[lambda][mu] = L_{parent, mu}(xi_{c, lambda})
  h.E.assign((size_t)ncl * P * P, 0.0);
  for (int c = 0; c < ncl; ++c) {
    const int par = h.cl[c].parent;
    if (par < 0) continue;
    const double* px = &h.nodes[((size_t)par * 3) * m];
    for (int l0 = 0; l0 < m; ++l0)
      for (int l1 = 0; l1 < m; ++l1)
        for (int l2 = 0; l2 < m; ++l2) {
          const double xi[3] = {h.nodes[((size_t)c * 3 + 0) * m + l0], h.nodes[((size_t)c * 3 + 1) * m + l1],
                                h.nodes[((size_t)c * 3 + 2) * m + l2]};
          const int lam = (l0 * m + l1) * m + l2;
          for (int a0 = 0; a0 < m; ++a0)
            for (int a1 = 0; a1 < m; ++a1)
              for (int a2 = 0; a2 < m; ++a2)
                h.E[((size_t)c * P + lam) * P + (a0 * m + a1) * m + a2] =
                    lagrange(px, m, a0, xi[0]) * lagrange(px + m, m, a1, xi[1]) * lagrange(px + 2 * m, m, a2, xi[2]);
        }
  }
  // block cluster tree: admissible blocks become far blocks, inadmissible
  // leaf pairs near blocks (sons(r) x sons(c), or one side fixed at a leaf)
  h.blocks.clear();
  std::function<void(int, int)> brec = [&](int r, int c) {
    const Cluster &R = h.cl[r], &Cc = h.cl[c];
    if (std::max(box_diam(R), box_diam(Cc)) <= p.opt.eta * box_dist(R, Cc)) {
      BlockDesc b{};
      b.r = r;
      b.c = c;
      b.kind = ((int64_t)R.size() * Cc.size() > (int64_t)P * P) ? kFarCore : kFarExpanded;
      b.rows = P;
      b.cols = P;
      h.blocks.push_back(b);
      return;
    }
    if (R.nsons == 0 && Cc.nsons == 0) {
      BlockDesc b{};
      b.r = r;
      b.c = c;
      b.kind = kNear;
      b.rows = R.size();
      b.cols = Cc.size();
      h.blocks.push_back(b);
      return;
    }
    const int nr = R.nsons ? 2 : 1, nc = Cc.nsons ? 2 : 1;
    for (int a = 0; a < nr; ++a)
      for (int bb = 0; bb < nc; ++bb) brec(R.nsons ? R.son[a] : r, Cc.nsons ? Cc.son[bb] : c);
  };
  brec(0, 0);
  // storage plan (Rcap slices per block; fibres for every system)
  const int R = h.Rcap;
  int64_t coff = 0, doff = 0;
  h.n_far = h.n_near = h.n_core = 0;
  std::vector<char> need_full(ncl, 0);
  for (auto& b : h.blocks) {
    if (b.kind == kNear) {
      b.arows = b.rows;
      b.acols = b.cols;
      ++h.n_near;
    } else {
      ++h.n_far;
      if (b.kind == kFarCore) {
        b.arows = b.acols = P;
        ++h.n_core;
        // time marching expands What_0 densely, cores through full bases
        if (p.opt.marching) need_full[b.r] = need_full[b.c] = 1;
      } else {
        b.arows = h.cl[b.r].size();
        b.acols = h.cl[b.c].size();
        need_full[b.r] = need_full[b.c] = 1;
      }
    }
    b.c_off = coff;
    coff += (int64_t)R * b.arows * b.acols;
    b.d_off = doff;
    doff += (int64_t)R * h.nsys;
  }
  h.cstore_elems = coff;
  h.dvec_elems = doff;
  // MACA batches bounded by a staging budget (cf64 elements): room for 512
  // of the largest block tensors at once (two workgroups per compute unit),
  // at least 2 GiB and at most 16 GiB unless one block needs more
  int64_t biggest = 0;
  for (auto& b : h.blocks) biggest = std::max<int64_t>(biggest, (int64_t)R * b.rows * b.cols);
  h.stage_budget = std::max<int64_t>(
      biggest, std::min<int64_t>((int64_t)1 << 30, std::max<int64_t>((int64_t)1 << 27, 512 * biggest)));
  h.batches.clear();
  int64_t acc = 0;
  int b0 = 0;
  for (int k = 0; k < (int)h.blocks.size(); ++k) {
    const int64_t need = (int64_t)R * h.blocks[k].rows * h.blocks[k].cols;
    if (acc + need > h.stage_budget) {
      h.batches.push_back({b0, k});
      b0 = k;
      acc = 0;
    }
    h.blocks[k].stage_off = acc;
    acc += need;
  }
  h.batches.push_back({b0, (int)h.blocks.size()});
  h.stage_elems = 0;
  for (auto& bt : h.batches) {
    int64_t s = 0;
    for (int k = bt.first; k < bt.second; ++k) s += (int64_t)R * h.blocks[k].rows * h.blocks[k].cols;
    h.stage_elems = std::max(h.stage_elems, s);
  }
  // full cluster bases of clusters used by expanded far blocks
  h.ufull_off.assign(ncl + 1, 0);
  for (int c = 0; c < ncl; ++c) h.ufull_off[c + 1] = h.ufull_off[c] + (need_full[c] ? (int64_t)h.cl[c].size() * P : 0);
  h.Ufull.assign(h.ufull_off.back(), 0.0);
  for (int c = 0; c < ncl; ++c)
    if (need_full[c]) basis_rows(c, &h.Ufull[h.ufull_off[c]]);
  // per-row-cluster lists of core blocks; per-leaf task lists
  h.core_by_row.assign(ncl, {});
  for (int k = 0; k < (int)h.blocks.size(); ++k)
    if (h.blocks[k].kind == kFarCore) h.core_by_row[h.blocks[k].r].push_back(k);
}

}  // namespace cqm
