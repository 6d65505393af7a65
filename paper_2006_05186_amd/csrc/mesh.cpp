// Mesh tables on the device: quadrature points, normals, near-field
// structure, cut-off boxes, CQM frequency tables, and the solve-workspace
// layout.  (The host-only planning -- quadrature rules, near-field
// adjacency -- is in planner.cpp.)
#include <algorithm>
#include <cmath>
#include <map>
#include <set>

#include "internal.h"
#include "fp64_math.h"

namespace cqm {

namespace {
template <typename T> T* upload(const std::vector<T>& h) {
  T* d = nullptr;
  if (h.empty()) return nullptr;
  CQM_HIP(hipMalloc(&d, sizeof(T) * h.size()));
  CQM_HIP(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return d;
}
}  // namespace

void upload_problem(Problem& p) {
  const int64_t M = p.M;
  double bary[6][3], w[6];
  dunavant6(bary, w);
  std::vector<double4> p64(M * kQ);
  std::vector<float4> p32(M * kQ);
  std::vector<int4> vid(M);
  std::vector<double> area(M);
  for (int64_t i = 0; i < M; ++i) {
    const double* A = &p.verts[3 * p.tris[3 * i]];
    const double* B = &p.verts[3 * p.tris[3 * i + 1]];
    const double* C = &p.verts[3 * p.tris[3 * i + 2]];
    const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
    const double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
    const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
                 cz = u[0] * v[1] - u[1] * v[0];
    area[i] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    for (int a = 0; a < kQ; ++a) {
      double q[3];
      for (int d = 0; d < 3; ++d) q[d] = bary[a][0] * A[d] + bary[a][1] * B[d] + bary[a][2] * C[d];
      p64[i * kQ + a] = double4{q[0], q[1], q[2], w[a] * area[i]};
      p32[i * kQ + a] = float4{(float)q[0], (float)q[1], (float)q[2], (float)(w[a] * area[i])};
    }
    vid[i] = int4{p.tris[3 * i], p.tris[3 * i + 1], p.tris[3 * i + 2], 0};
  }
  p.dev.pts64 = upload(p64);
  p.dev.pts32 = upload(p32);
  {
    // unit normals in the triangles' vertex order (the double-layer kernel)
    std::vector<double4> nrm(M);
    for (int64_t i = 0; i < M; ++i) {
      const double* A = &p.verts[3 * p.tris[3 * i]];
      const double* B = &p.verts[3 * p.tris[3 * i + 1]];
      const double* C = &p.verts[3 * p.tris[3 * i + 2]];
      const double u[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      const double v[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
      const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2],
                           u[0] * v[1] - u[1] * v[0]};
      const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      nrm[i] = double4{n[0] / nn, n[1] / nn, n[2] / nn, 0.0};
    }
    p.dev.nrm64 = upload(nrm);
  }
  {
    // bounding boxes of the triangles of each 64-block and 16-group (the
    // vertex boxes contain every quadrature point), for the cut-off
    auto boxes = [&](int g) {
      const int64_t nb = (M + g - 1) / g;
      std::vector<double> b(nb * 6);
      for (int64_t k = 0; k < nb; ++k) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t i = k * g; i < std::min<int64_t>(M, (k + 1) * g); ++i)
          for (int v = 0; v < 3; ++v)
            for (int d = 0; d < 3; ++d) {
              const double x = p.verts[3 * p.tris[3 * i + v] + d];
              lo[d] = std::min(lo[d], x);
              hi[d] = std::max(hi[d], x);
            }
        for (int d = 0; d < 3; ++d) b[6 * k + d] = lo[d], b[6 * k + 3 + d] = hi[d];
      }
      return b;
    };
    const std::vector<double> b64 = boxes(kSymB), b16 = boxes(16);
    const int nb = sym_blocks((int)M);
    std::vector<float> gap((size_t)sym_tiles((int)M));
    for (int J = 0; J < nb; ++J)
      for (int I = 0; I <= J; ++I) {
        double g2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double gd = std::max(0.0, std::max(b64[6 * I + d] - b64[6 * J + 3 + d],
                                                   b64[6 * J + d] - b64[6 * I + 3 + d]));
          g2 += gd * gd;
        }
        // rounded down so the float never exceeds the true gap
        gap[(size_t)J * (J + 1) / 2 + I] = std::nextafter((float)std::sqrt(g2), 0.0f);
      }
    p.dev.tile_gap = upload(gap);
    p.tile_gap_host = gap;
    p.dev.sub_box = upload(b16);
  }
  p.dev.vid = upload(vid);
  p.dev.area = upload(area);
  p.dev.verts = upload(p.verts);
  p.dev.near_rowptr = upload(p.rowptr);
  p.dev.near_col = upload(p.col);
  std::vector<int32_t> krow(p.col.size());
  for (int64_t i = 0; i < M; ++i)
    for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) krow[k] = (int32_t)i;
  p.dev.near_row = upload(krow);
  p.dev.near_kind = upload(p.kind);
  p.dev.near_vtx = upload(p.nvtx);
  {
    // position of pair (j, i) for every pair (i, j) (the pattern is
    // symmetric: sharing a vertex is)
    std::vector<int32_t> tpos(p.col.size());
    for (int64_t i = 0; i < M; ++i)
      for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k) {
        const int j = p.col[k];
        const int32_t* b = p.col.data() + p.rowptr[j];
        const int32_t* e = p.col.data() + p.rowptr[j + 1];
        const int32_t* f = std::lower_bound(b, e, (int32_t)i);
        require(f != e && *f == i, CQM_EINVAL, "near-field pattern is not symmetric");
        tpos[k] = (int32_t)(f - p.col.data());
      }
    p.dev.near_tpos = upload(tpos);
  }
  CQM_HIP(hipMalloc(&p.dev.near_static, sizeof(double) * std::max<size_t>(1, p.col.size())));
  CQM_HIP(hipMalloc(&p.dev.nearK_static, sizeof(double) * std::max<size_t>(1, p.col.size())));
  if (p.opt.formulation == CQM_FORMULATION_DIRECT)
    CQM_HIP(hipMalloc(&p.dev.nearD_static, sizeof(double) * 9 * std::max<size_t>(1, p.col.size())));
  {
    // vertex -> (triangle, local vertex) slots, ascending: the fixed order
    // in which the hypersingular product sums a vertex's contributions
    std::vector<int32_t> ptr(p.nv + 1, 0), slot(3 * M);
    for (int64_t k = 0; k < 3 * M; ++k) ++ptr[p.tris[k] + 1];
    for (int64_t v = 0; v < p.nv; ++v) ptr[v + 1] += ptr[v];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t k = 0; k < 3 * M; ++k) slot[fill[p.tris[k]]++] = (int32_t)k;
    p.dev.v2t_ptr = upload(ptr);
    p.dev.v2t = upload(slot);
  }
  std::vector<double> gx, gw;
  gauss_legendre01(p.opt.q_duffy, gx, gw);
  std::vector<double> gl(gx);
  gl.insert(gl.end(), gw.begin(), gw.end());
  p.dev.gl = upload(gl);
  // frequency tables
  const int F = p.F;
  std::vector<cf64> s(F), twf(F), twi(F);
  std::vector<double> rp(F), rip(F);
  for (int l = 0; l < F; ++l) s[l] = cf64{p.s_re[l], p.s_im[l]};
  for (int k = 0; k <= F / 2; ++k) {
    const double c = std::cos(2.0 * M_PI * k / F), sn = std::sin(2.0 * M_PI * k / F);
    twf[k] = cf64{c, -sn};
    twi[k] = cf64{c, sn};
    if (k > 0) {
      twf[F - k] = cf64{c, sn};
      twi[F - k] = cf64{c, -sn};
    }
  }
  for (int n = 0; n < F; ++n) {
    rp[n] = std::pow(p.rho, n);
    rip[n] = std::pow(p.rho, -n) / F;
  }
  p.dev.s = upload(s);
  p.dev.tw_fwd = upload(twf);
  p.dev.tw_inv = upload(twi);
  p.dev.rho_pow = upload(rp);
  p.dev.rho_ipow = upload(rip);
  std::vector<double> ea64(F), pb64(F);
  std::vector<float> ea32(F), pb32(F);
  const double log2e = 1.4426950408889634;
  for (int l = 0; l < F; ++l) {
    ea64[l] = -p.s_re[l];
    pb64[l] = p.s_im[l];
    ea32[l] = (float)(-p.s_re[l] * log2e);
    pb32[l] = (float)(p.s_im[l] / (2.0 * M_PI));
  }
  p.dev.ea64 = upload(ea64);
  p.dev.pb64 = upload(pb64);
  // the same coefficients in table steps (256/ln2 and 512/(2 pi) per unit:
  // the dense assembly's exponential and fine sine/cosine tables)
  {
    std::vector<double> eu(F), pu(F);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const long double ln2 = 0.693147180559945309417232121458176568L;
    for (int l = 0; l < F; ++l) {
      eu[l] = (double)((long double)ea64[l] * 256.0L / ln2);
      pu[l] = (double)((long double)pb64[l] * 512.0L / two_pi);
    }
    p.dev.ea64u = upload(eu);
    p.dev.pb64u = upload(pu);
  }
  // tables of the FP64 exp/sincos (extended precision, rounded once)
  std::vector<double> ftab(kFp64TabTotal);
  const long double pi_l = 3.141592653589793238462643383279502884L;
  for (int j = 0; j < 256; ++j) {
    ftab[j] = (double)std::exp2((long double)j / 256.0L);
    ftab[256 + 2 * j] = (double)std::sin(pi_l * j / 128.0L);
    ftab[256 + 2 * j + 1] = (double)std::cos(pi_l * j / 128.0L);
  }
  for (int j = 0; j < 512; ++j) {
    ftab[kFp64Tab512Off + 2 * j] = (double)std::sin(pi_l * j / 256.0L);
    ftab[kFp64Tab512Off + 2 * j + 1] = (double)std::cos(pi_l * j / 256.0L);
  }
  p.dev.ftab = upload(ftab);
  p.dev.ea32 = upload(ea32);
  p.dev.pb32 = upload(pb32);
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool mode_is_mixed(int mode) { return mode == CQM_MIXED_PLAIN || mode == CQM_MIXED_H2ACA; }
bool mode_is_h2(int mode) { return mode == CQM_MIXED_H2ACA || mode == CQM_FP64_H2ACA; }

size_t h2_workspace_bytes(const Problem& p);  // h2.cpp

size_t state_layout(const Problem& p, SolveState& st) {
  const size_t M = p.M, Fs = p.Fsys, m = p.opt.gmres_restart;
  const size_t inner = mode_is_mixed(p.opt.mode) ? sizeof(cf32) : sizeof(cf64);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  st.b = take(sizeof(double) * p.F * M);
  st.ghat = take(sizeof(cf64) * Fs * M);
  st.x = take(sizeof(cf64) * Fs * M);
  st.r = take(sizeof(cf64) * Fs * M);
  st.basis = take(inner * Fs * (m + 1) * M);
  st.H = take(sizeof(cf64) * Fs * (m + 1) * m);
  st.cs = take(sizeof(double) * Fs * m);
  st.sn = take(sizeof(cf64) * Fs * m);
  st.g = take(sizeof(cf64) * Fs * (m + 1));
  st.sysd = take(sizeof(double) * 8 * Fs);
  st.sysi = take(sizeof(int) * kSysiStride * Fs);
  st.part = take(sizeof(double) * Fs * ((M + kArnRows - 1) / kArnRows) * (4 * (m + 1) + 2));
  // tile partial sums of stored-operator products (sized for the
  // double-double residual: (hi, lo) pairs of FP64 complex values)
  const bool stored = !mode_is_h2(p.opt.mode) && p.opt.form == CQM_FORM_DENSE;
  st.sym = stored ? take(2 * sizeof(cf64) * Fs * sym_partials((int)M)) : 0;
  st.scratch = take(4096);
  st.total = off;
  return off;
}

void compute_layout(Problem& p) {
  Layout L;
  const size_t M = p.M, Fs = p.Fsys;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  // the problem's own solve state first, then the operator
  p.own.p = &p;
  off = state_layout(p, p.own);
  if (mode_is_h2(p.opt.mode)) {
    L.partial = take(h2_workspace_bytes(p));
    const bool bj = p.opt.precond == CQM_PRECOND_BLOCK_JACOBI;
    // block-Jacobi and the plain refinement residual both need the plain
    // operator's near-field values
    if (bj || p.opt.refine_plain)
      L.near_val = take(sizeof(cf64) * Fs * std::max<size_t>(1, p.col.size()));
    if (bj) {
      // block-Jacobi from the plain operator's diagonal blocks (FP64,
      // compact) and their inverses
      L.diag64 = take(sizeof(cf64) * Fs * block_inverse_elems((int)M));
      L.pinv = take((mode_is_mixed(p.opt.mode) ? sizeof(cf32) : sizeof(cf64)) * Fs *
                    block_inverse_elems((int)M));
    }
    if (p.opt.refine_plain) {
      // partial sums of the FP64 matrix-free product (every system at once)
      size_t worst = 0;
      for (int nl = 1; nl <= (int)Fs; ++nl)
        worst = std::max(worst, (size_t)far_partial_slots((int)M, nl, 64) * nl * sizeof(cf64));
      L.mfpart = take(worst * M);
    }
  } else {
    L.near_val = take(sizeof(cf64) * Fs * std::max<size_t>(1, p.col.size()));
    if (p.opt.form == CQM_FORM_DENSE) {
      L.dense64 = take(sizeof(cf64) * Fs * sym_slice((int)M));
      if (mode_is_mixed(p.opt.mode)) L.dense32 = take(sizeof(cf32) * Fs * sym_slice((int)M));
      if (p.opt.precond == CQM_PRECOND_BLOCK_JACOBI)
        L.pinv = take((mode_is_mixed(p.opt.mode) ? sizeof(cf32) : sizeof(cf64)) * Fs *
                      block_inverse_elems((int)M));
    } else {
      size_t worst = 0;
      for (int nl = 1; nl <= (int)Fs; ++nl) {
        const size_t a = (size_t)far_partial_slots((int)M, nl, 32) * nl * sizeof(cf32);
        const size_t b = (size_t)far_partial_slots((int)M, nl, 64) * nl * sizeof(cf64);
        worst = std::max(worst, std::max(a, b));
      }
      L.partial = take(worst * M);
      if (p.opt.precond == CQM_PRECOND_BLOCK_JACOBI) {
        // the diagonal blocks (FP64, compact) and their inverses
        L.diag64 = take(sizeof(cf64) * Fs * block_inverse_elems((int)M));
        L.pinv = take((mode_is_mixed(p.opt.mode) ? sizeof(cf32) : sizeof(cf64)) * Fs *
                      block_inverse_elems((int)M));
      }
    }
  }
  if (p.opt.marching && !mode_is_h2(p.opt.mode) && p.opt.form == CQM_FORM_DENSE) {
    // time marching: N+1 real weight slices, the block inverses of What_0
    // (and their complex staging), the history product's partial slots and
    // the CG vectors with their per-workgroup partials
    const int Mi = (int)M, nb = sym_blocks(Mi);
    const size_t nwg = (M + 255) / 256;
    L.mchunks = march_chunks(Mi, std::max(1, p.N));
    L.mw = take(sizeof(double) * p.F * sym_slice(Mi));
    L.mpinv = take(sizeof(cf64) * block_inverse_elems(Mi));
    L.mdiag = take(sizeof(cf64) * block_inverse_elems(Mi));
    L.mpart = take(sizeof(double) * L.mchunks * (size_t)nb * nb * kSymB);
    L.mvec = take(sizeof(double) * (5 * M + 5 * nwg) + 256);
  }
  if (p.opt.marching && mode_is_h2(p.opt.mode)) {
    // compressed time marching (weights from the fibres, in the compressed
    // operator's own workspace): the past densities in cluster order, the
    // history sum, the CG product's vectors and vectors/partials, the block
    // inverses of What_0
    const size_t nwg = (M + 255) / 256;
    L.mz = take(sizeof(cf64) * p.F * M);
    L.my = take(sizeof(cf64) * M);
    L.mpc = take(sizeof(cf64) * 2 * M);
    L.mpinv = take(sizeof(cf64) * block_inverse_elems((int)M));
    L.mdiag = take(sizeof(cf64) * block_inverse_elems((int)M));
    L.mvec = take(sizeof(double) * (5 * M + 5 * nwg) + 256);
  }
  if (p.opt.formulation == CQM_FORMULATION_DIRECT) {
    // double-layer operator for the direct right-hand side
    L.nearK = take(sizeof(cf64) * Fs * std::max<size_t>(1, p.col.size()));
    L.kin = take(sizeof(cf64) * Fs * M);
    L.kpart = take(dl_partial_bytes((int)M, (int)Fs));
    // hypersingular product: per-triangle sources, partial sums, slots
    L.dsrc = take(sizeof(cf64) * 9 * Fs * M);
    L.dpart = take(hs_partial_bytes((int)M, (int)Fs));
    L.dz = take(sizeof(cf64) * 3 * Fs * M);
  }
  L.total = off;
  p.lay = L;
}

}  // namespace cqm
