// Solve driver: operator preparation, right-hand sides and transforms, and
// the batched restarted-GMRES engine with FP64 refinement over any set of
// solve states (one problem, an uneven batch, or the serving loop's active
// requests).
#include <algorithm>
#include <cstring>
#include <memory>
#include <chrono>
#include <cmath>
#include <map>

#include "internal.h"

namespace cqm {
void h2_prepare(Problem& p, hipStream_t s);
template <typename R>
void h2_apply(Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
              const int* active, hipStream_t s);
void h2_stats(const Problem& p, cqm_diag* d);

namespace {
template <typename T> T* wsp(Problem& p, size_t off) { return reinterpret_cast<T*>(p.ws + off); }
double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}
template <typename T> void ensure(T*& ptr, size_t& cap, size_t n) {
  if (n <= cap && ptr) return;
  if (ptr) CQM_HIP(hipFree(ptr));
  ptr = nullptr;
  const size_t c = std::max<size_t>(n, 2 * cap);
  CQM_HIP(hipMalloc(&ptr, sizeof(T) * c));
  cap = c;
}
bool dense_form(const Problem& p) { return !mode_is_h2(p.opt.mode) && p.opt.form == CQM_FORM_DENSE; }

// Entries of the stored upper triangle a product reads per frequency under
// the inner and the FP64 cut-off (from the host copy of the tile gaps),
// once per problem.
void cut_entries(Problem& p) {
  if ((int)p.cut_entries32.size() == p.Fsys) return;
  const int M = (int)p.M, nb = sym_blocks(M);
  const std::vector<float>& gap = p.tile_gap_host;
  p.cut_entries32.assign(p.Fsys, 0);
  p.cut_entries64.assign(p.Fsys, 0);
  for (int l = 0; l < p.Fsys; ++l) {
    const float c32 = std::nextafter(cutoff_radius(p.opt.cutoff_inner, p.s_re[l]), 3.4e38f);
    const float c64 = std::nextafter(cutoff_radius(p.opt.cutoff_outer, p.s_re[l]), 3.4e38f);
    for (int J = 0; J < nb; ++J)
      for (int I = 0; I <= J; ++I) {
        const int64_t ri = std::min(kSymB, M - I * kSymB), cj = std::min(kSymB, M - J * kSymB);
        const int64_t e = I == J ? ri * (ri + 1) / 2 : ri * cj;
        const float g = gap[(size_t)J * (J + 1) / 2 + I];
        if (!(g >= c32)) p.cut_entries32[l] += e;
        if (!(g >= c64)) p.cut_entries64[l] += e;
      }
  }
}
}  // namespace

// The plain operator without a stored copy: far-field kernel evaluation on
// the fly plus the near-field values (Section 3.2).  The matrix-free form's
// product, and the refinement residual of compressed problems with
// refine_plain (their partial sums have a buffer of their own, the
// compressed operator occupying the matrix-free form's).
template <typename R>
void apply_plain_free(Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y,
                      int64_t ys, const int* active, hipStream_t s) {
  const size_t off = mode_is_h2(p.opt.mode) ? p.lay.mfpart : p.lay.partial;
  require(off != 0 && p.lay.near_val != 0, CQM_EINVAL, "no buffers for the matrix-free product");
  cplx<R>* partial = wsp<cplx<R>>(p, off);
  {
    const int c = sizeof(R) == 4 ? CQM_K_FAR32 : CQM_K_FAR64;
    Timed t(p, c, s);
    launch_far_apply<R>(p, l0, nsys, x, xs, partial, active, p.timer.ctr(c), s);
  }
  Timed t(p, CQM_K_NEAR, s);
  launch_far_reduce_near<R>(p, l0, nsys, partial, x, xs, y, ys, wsp<cf64>(p, p.lay.near_val),
                            active, s);
}

template <typename R>
void apply_op(Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
              const int* active, hipStream_t s) {
  if (mode_is_h2(p.opt.mode)) {
    Timed t(p, sizeof(R) == 4 ? CQM_K_GEMV32 : CQM_K_GEMV64, s);
    h2_apply<R>(p, l0, nsys, x, xs, y, ys, active, s);
    return;
  }
  if (p.opt.form != CQM_FORM_DENSE) {
    apply_plain_free<R>(p, l0, nsys, x, xs, y, ys, active, s);
    return;
  }
  const int M = (int)p.M;
  const cplx<R>* V;
  if constexpr (sizeof(R) == 4) {
    require(p.lay.dense32 != 0, CQM_EINVAL, "FP32 dense operator exists only in mixed mode");
    V = wsp<cf32>(p, p.lay.dense32);
  } else {
    V = wsp<cf64>(p, p.lay.dense64);
  }
  require(p.own.sym != 0, CQM_EINVAL, "no partial-sum buffer for the stored operator");
  Timed t(p, sizeof(R) == 4 ? CQM_K_GEMV32 : CQM_K_GEMV64, s);
  launch_dense_gemv<R>(V + (int64_t)l0 * sym_slice(M), M, nsys, x, xs, y, ys, active,
                       p.own.at<cplx<R>>(p.own.sym), s);
}
template void apply_op<float>(Problem&, int, int, const cf32*, int64_t, cf32*, int64_t, const int*, hipStream_t);
template void apply_op<double>(Problem&, int, int, const cf64*, int64_t, cf64*, int64_t, const int*, hipStream_t);

// Block-Jacobi inverses of the matrix-free and compressed forms: the plain
// operator's diagonal blocks assembled on their own (near pairs from nv),
// then inverted.
static void diag_block_inverses(Problem& p, const cf64* nv, hipStream_t s) {
  cf64* dg = wsp<cf64>(p, p.lay.diag64);
  {
    Timed t(p, CQM_K_ASSEMBLE, s);
    launch_diag_blocks(p, dg, nv, s);
  }
  Timed t(p, CQM_K_OTHER, s);
  if (mode_is_mixed(p.opt.mode)) launch_block_inverse<float>(dg, (int)p.M, p.Fsys, true, wsp<cf32>(p, p.lay.pinv), s);
  else launch_block_inverse<double>(dg, (int)p.M, p.Fsys, true, wsp<cf64>(p, p.lay.pinv), s);
}

// Block-Jacobi inverses of an assembled stored operator, and its ready flag.
static void finish_dense(Problem& p, hipStream_t s) {
  if (p.lay.pinv) {
    cf64* d64 = wsp<cf64>(p, p.lay.dense64);
    Timed t(p, CQM_K_OTHER, s);
    if (mode_is_mixed(p.opt.mode)) launch_block_inverse<float>(d64, (int)p.M, p.Fsys, false, wsp<cf32>(p, p.lay.pinv), s);
    else launch_block_inverse<double>(d64, (int)p.M, p.Fsys, false, wsp<cf64>(p, p.lay.pinv), s);
  }
  p.dense_ready = true;
}

// Near field and (dense form) the assembled operator, or the compressed one.
// With defer_dense, a stored-form operator that needs assembling is left to
// the caller (returns true: assemble, then finish_dense).
static bool prepare_operator_impl(Problem& p, hipStream_t s, bool defer_dense);
void prepare_operator(Problem& p, hipStream_t s) { prepare_operator_impl(p, s, false); }

// Near values of the double-layer operator (direct formulation): the static
// part once per mesh, the per-frequency values once per operator.
void prepare_double_layer(Problem& p, hipStream_t s) {
  require(p.lay.nearK != 0, CQM_EINVAL, "no double-layer buffers (formulation is not DIRECT)");
  Timed t(p, CQM_K_NEAR, s);
  if (!p.nearK_static_ready) {
    launch_nearK_static(p, s);
    p.nearK_static_ready = true;
  }
  if (!(p.nearK_ready && p.opt.reuse_operator)) {
    launch_nearK_values(p, wsp<cf64>(p, p.lay.nearK), s);
    p.nearK_ready = true;
  }
}

static bool prepare_operator_impl(Problem& p, hipStream_t s, bool defer_dense) {
  Stage stage("prepare_operator");
  require(p.ws != nullptr, CQM_ENOMEM, "no workspace attached (cqm_set_workspace)");
  if (p.opt.formulation == CQM_FORMULATION_DIRECT) prepare_double_layer(p, s);
  if (!p.static_ready) {
    Timed t(p, CQM_K_NEAR, s);
    launch_near_static(p, s);
    p.static_ready = true;
  }
  if (mode_is_h2(p.opt.mode)) {
    if (!(p.opt.reuse_operator && p.near_ready)) {
      {
        Timed t(p, CQM_K_ASSEMBLE, s);
        h2_prepare(p, s);
      }
      if (p.lay.near_val) {
        cf64* nv = wsp<cf64>(p, p.lay.near_val);
        {
          Timed t(p, CQM_K_NEAR, s);
          launch_near_values(p, nv, s);
        }
        if (p.lay.pinv) diag_block_inverses(p, nv, s);
      }
    }
    p.near_ready = true;
    return false;
  }
  const bool have = p.near_ready && (p.opt.form != CQM_FORM_DENSE || p.dense_ready);
  if (have && p.opt.reuse_operator) return false;
  cf64* nv = wsp<cf64>(p, p.lay.near_val);
  {
    Timed t(p, CQM_K_NEAR, s);
    launch_near_values(p, nv, s);
  }
  p.near_ready = true;
  if (p.opt.form == CQM_FORM_MATRIX_FREE && p.lay.pinv) diag_block_inverses(p, nv, s);
  if (p.opt.form == CQM_FORM_DENSE) {
    p.dense_ready = false;
    if (defer_dense) return true;
    cf64* d64 = wsp<cf64>(p, p.lay.dense64);
    cf32* d32 = p.lay.dense32 ? wsp<cf32>(p, p.lay.dense32) : nullptr;
    {
      Timed t(p, CQM_K_ASSEMBLE, s);
      launch_dense_assemble(p, d64, d32, nv, p.timer.ctr(CQM_K_ASSEMBLE), s);
    }
    finish_dense(p, s);
  }
  return false;
}

// Operators of a batch: near fields per problem, then every stored operator
// that needs assembling in one work-queue launch, then their block inverses.
static void prepare_batch(std::vector<SolveState*>& G, hipStream_t s) {
  std::vector<Problem*> ps;
  std::vector<cf64*> d64;
  std::vector<cf32*> d32;
  std::vector<const cf64*> nv;
  for (SolveState* st : G) {
    Problem& p = *st->p;
    CQM_HIP(hipSetDevice(p.ctx->device));
    require(p.ws != nullptr && p.ws_bytes >= p.lay.total, CQM_ENOMEM,
            "workspace missing or smaller than cqm_workspace_size");
    if (std::find(ps.begin(), ps.end(), &p) != ps.end()) continue;
    if (prepare_operator_impl(p, s, true)) {
      ps.push_back(&p);
      d64.push_back(wsp<cf64>(p, p.lay.dense64));
      d32.push_back(p.lay.dense32 ? wsp<cf32>(p, p.lay.dense32) : nullptr);
      nv.push_back(wsp<cf64>(p, p.lay.near_val));
    }
  }
  if (ps.empty()) return;
  Problem& p0 = *G[0]->p;
  {
    Timed t(p0, CQM_K_ASSEMBLE, s);
    launch_dense_assemble_batch(ps, d64, d32, nv, p0.timer.ctr(CQM_K_ASSEMBLE), s);
  }
  for (Problem* p : ps) finish_dense(*p, s);
}

// Operator (optionally), right-hand side and forward transform of one state.
void pre_solve(SolveState& st, hipStream_t s, bool prepare, bool timed) {
  Stage stage("operator_and_right_hand_side");
  Problem& p = *st.p;
  CQM_HIP(hipSetDevice(p.ctx->device));
  require(p.ws != nullptr && p.ws_bytes >= p.lay.total, CQM_ENOMEM,
          "workspace missing or smaller than cqm_workspace_size");
  require(st.inc.kind != 0, CQM_EINVAL, "no incident data set");
  require(st.q_out != nullptr, CQM_EINVAL, "q_out is NULL");
  st.diag = cqm_diag{};
  if (prepare && timed) {
    // GPU time of the setup, read after the solve's closing synchronisation
    for (hipEvent_t& e : p.setup_ev)
      if (!e) CQM_HIP(hipEventCreate(&e));
    CQM_HIP(hipEventRecord(p.setup_ev[0], s));
    prepare_operator(p, s);
    CQM_HIP(hipEventRecord(p.setup_ev[1], s));
    st.diag.t_setup_ms = -1.0;  // pending
  } else if (prepare) {
    auto t0 = std::chrono::steady_clock::now();
    prepare_operator(p, s);
    CQM_HIP(hipStreamSynchronize(s));
    st.diag.t_setup_ms = ms_since(t0);
  }
  {
    Timed t(p, CQM_K_OTHER, s);
    launch_rhs(p, st.inc, st.at<double>(st.b), s);
    launch_dft_forward(p, st.at<double>(st.b), st.at<cf64>(st.ghat), st.at<double>(st.scratch), s);
  }
  if (p.opt.formulation == CQM_FORMULATION_DIRECT) {
    // direct formulation: ghat_l = -1/2 ghat_l + K_l (ghat_l / area), the
    // transforms of <phi_i, (-1/2 I + K) g_D> with g_D's piecewise-constant
    // coefficients b_n / area
    if (!p.nearK_ready) prepare_double_layer(p, s);
    const int M = (int)p.M;
    cf64* g = st.at<cf64>(st.ghat);
    cf64* c = wsp<cf64>(p, p.lay.kin);
    Timed t(p, CQM_K_FAR64, s);
    launch_div_area(p, p.Fsys, g, M, c, s);
    launch_apply_K(p, 0, p.Fsys, c, M, g, -0.5, g, M, wsp<cf64>(p, p.lay.nearK),
                   wsp<cf64>(p, p.lay.kpart), false, s);
  }
}

// Inverse transform and operator diagnostics of one state.
void post_solve(SolveState& st, hipStream_t s) {
  Stage stage("inverse_transform");
  Problem& p = *st.p;
  cqm_diag& dg = st.diag;
  double* sums = st.at<double>(st.scratch);  // cleared by the forward transform
  {
    Timed t(p, CQM_K_OTHER, s);
    launch_dft_inverse(p, st.at<cf64>(st.x), st.q_out, sums, sums + 1, s);
  }
  double hs[2];
  CQM_HIP(hipMemcpyAsync(hs, sums, sizeof(hs), hipMemcpyDeviceToHost, s));
  CQM_HIP(hipStreamSynchronize(s));
  if (dg.t_setup_ms < 0.0) {
    float ms = 0.f;
    CQM_HIP(hipEventElapsedTime(&ms, p.setup_ev[0], p.setup_ev[1]));
    dg.t_setup_ms = ms;
  }
  dg.imag_ratio = p.full_band() && hs[1] > 0 ? std::sqrt(hs[0] / hs[1]) : 0.0;
  dg.n_systems = p.Fsys;
  dg.far_units = p.far_units;
  if (!mode_is_h2(p.opt.mode) && p.opt.form == CQM_FORM_MATRIX_FREE) {
    const FarShape sh = far_shape_of(p, p.Fsys, mode_is_mixed(p.opt.mode) ? 32 : 64);
    dg.far_tile = sh.ft;
    dg.far_waves = sh.waves;
  }
  if (mode_is_h2(p.opt.mode)) h2_stats(p, &dg);
  else if (p.opt.form == CQM_FORM_DENSE)
    dg.operator_bytes = (int64_t)p.Fsys * sym_slice((int)p.M) * (p.lay.dense32 ? 24 : 16);
  else
    dg.operator_bytes = (int64_t)p.Fsys * (int64_t)p.col.size() * 16;
}

int diag_status(const cqm_diag& dg) {
  if (dg.converged < 0) return CQM_ENAN;
  if (!dg.converged) return CQM_ENOCONV;
  return CQM_OK;
}

// ------------------------------------------------------------ engine
// Systems per batch below which the Arnoldi step is split over row slices
// (256 compute units: one workgroup per system leaves most of them idle).
constexpr int kSplitBelow = 256;

void Engine::set(const std::vector<SolveState*>& S, hipStream_t s) {
  S_ = S;
  hd_.clear();
  lite_.clear();
  groups_.clear();
  std::map<const void*, int> slot;
  maxM_ = 0;
  if (S_.empty()) return;
  m_ = S_[0]->p->opt.gmres_restart;
  mixed = mode_is_mixed(S_[0]->p->opt.mode);
  pre_ = false;
  anypre_ = false;
  bool pre_set = false;
  for (size_t k = 0; k < S_.size(); ++k) {
    SolveState* st = S_[k];
    Problem& p = *st->p;
    require(p.opt.gmres_restart == m_, CQM_EINVAL, "batched problems must share gmres_restart");
    require(mode_is_mixed(p.opt.mode) == mixed, CQM_EINVAL, "batched problems must share precision");
    const int M = (int)p.M;
    maxM_ = std::max(maxM_, M);
    st->first = (int)hd_.size();
    if (dense_form(p)) {
      // one Krylov layout for every stored-operator system of the batch
      const bool pk = p.lay.pinv != 0;
      require(!pre_set || pk == pre_, CQM_EINVAL,
              "batched stored-operator problems must share the preconditioner");
      pre_ = pk;
      pre_set = true;
    }
    const size_t isz = mixed ? sizeof(cf32) : sizeof(cf64);
    for (int l = 0; l < p.Fsys; ++l) {
      SysDesc d{};
      d.M = M;
      d.m = m_;
      d.prob = (int)k;
      d.l = l;
      d.basis = st->base + st->basis + isz * (size_t)l * (m_ + 1) * M;
      d.H = st->at<cf64>(st->H) + (size_t)l * (m_ + 1) * m_;
      d.cs = st->at<double>(st->cs) + (size_t)l * m_;
      d.sn = st->at<cf64>(st->sn) + (size_t)l * m_;
      d.g = st->at<cf64>(st->g) + (size_t)l * (m_ + 1);
      d.sysd = st->at<double>(st->sysd) + 8 * l;
      d.sysi = st->at<int>(st->sysi) + kSysiStride * l;
      d.x = st->at<cf64>(st->x) + (size_t)l * M;
      d.r = st->at<cf64>(st->r) + (size_t)l * M;
      d.ghat = st->at<cf64>(st->ghat) + (size_t)l * M;
      d.part = st->at<double>(st->part) + (size_t)l * ((M + kArnRows - 1) / kArnRows) * (4 * (m_ + 1) + 2);
      if (!dense_form(p) && p.lay.pinv) {
        // matrix-free and compressed forms: P v_j is formed in r's memory
        // (the product reads it and writes basis slot j + 1)
        d.Pinv = mixed ? (const void*)(wsp<cf32>(p, p.lay.pinv) + (size_t)l * block_inverse_elems(M))
                       : (const void*)(wsp<cf64>(p, p.lay.pinv) + (size_t)l * block_inverse_elems(M));
        d.zb = d.r;
        anypre_ = true;
      }
      if (dense_form(p)) {
        d.V64 = wsp<cf64>(p, p.lay.dense64) + (size_t)l * sym_slice(M);
        d.V32 = p.lay.dense32 ? (const void*)(wsp<cf32>(p, p.lay.dense32) + (size_t)l * sym_slice(M)) : nullptr;
        d.symp = st->base + st->sym + 2 * sizeof(cf64) * (size_t)l * sym_partials(M);
        if (p.lay.pinv) {
          d.Pinv = mixed ? (const void*)(wsp<cf32>(p, p.lay.pinv) + (size_t)l * block_inverse_elems(M))
                         : (const void*)(wsp<cf64>(p, p.lay.pinv) + (size_t)l * block_inverse_elems(M));
          anypre_ = true;
        }
        // join the group of systems on the same operator slice, if any
        auto it = slot.find(d.V64);
        if (it == slot.end() || groups_[it->second].n == kMaxGroup) {
          GemvGroup g{};
          g.n = 0;
          slot[d.V64] = (int)groups_.size();
          groups_.push_back(g);
          GroupLite gl{};
          gl.V32 = d.V32;
          gl.V64 = d.V64;
          gl.M = M;
          // cut-off radii of this frequency (rounded up: a skipped tile's
          // entries were all left out by the assembly)
          gl.gap = p.dev.tile_gap;
          gl.cut32 = std::nextafter(cutoff_radius(p.opt.cutoff_inner, p.s_re[l]), 3.4e38f);
          gl.cut64 = std::nextafter(cutoff_radius(p.opt.cutoff_outer, p.s_re[l]), 3.4e38f);
          cut_entries(p);
          gl.entries32 = p.cut_entries32[l];
          gl.entries64 = p.cut_entries64[l];
          lite_.push_back(gl);
          it = slot.find(d.V64);
        }
        GemvGroup& g = groups_[it->second];
        GroupLite& gl = lite_[it->second];
        gl.basis[g.n] = d.basis;
        gl.x[g.n] = d.x;
        gl.symp[g.n] = d.symp;
        gl.sysi[g.n] = d.sysi;
        g.sys[g.n++] = (int)hd_.size();
        gl.n = g.n;
      }
      hd_.push_back(d);
    }
  }
  const int n = (int)hd_.size();
  // split the Arnoldi step over row slices when one workgroup per system
  // would leave most compute units idle
  const int lay = S_[0]->p->opt.arnoldi_layout;
  split_ = lay == CQM_ARNOLDI_SPLIT || (lay == CQM_ARNOLDI_AUTO && n < kSplitBelow);
  const SysDesc* old_desc = eb.desc;
  ensure(eb.desc, eb.desc_cap, hd_.size());
  if (eb.desc != old_desc) drop_graphs();  // captured steps point at the old buffer
  ensure(eb.open_cycle, eb.cycle_cap, std::max<size_t>(1, lite_.size()));
  ensure(eb.open_step, eb.step_cap, std::max<size_t>(1, lite_.size()));
  if (eb.staging_cap < 2 * lite_.size()) {
    if (eb.staging) {
      CQM_HIP(hipStreamSynchronize(s));
      CQM_HIP(hipHostFree(eb.staging));
    }
    eb.staging = nullptr;
    eb.staging_cap = 0;
    const size_t c = std::max<size_t>(2 * lite_.size(), 256);
    CQM_HIP(hipHostMalloc((void**)&eb.staging, sizeof(GroupLite) * c, hipHostMallocDefault));
    eb.staging_cap = c;
  }
  ensure(eb.arn_desc, eb.arn_cap, std::max<size_t>(1, hd_.size()));
  if (eb.arn_staging_cap < 2 * (size_t)n) {
    if (eb.arn_staging) {
      CQM_HIP(hipStreamSynchronize(s));
      CQM_HIP(hipHostFree(eb.arn_staging));
    }
    eb.arn_staging = nullptr;
    eb.arn_staging_cap = 0;
    const size_t c = std::max<size_t>(2 * (size_t)n, 256);
    CQM_HIP(hipHostMalloc((void**)&eb.arn_staging, sizeof(SysDesc) * c, hipHostMallocDefault));
    eb.arn_staging_cap = c;
  }
  if (eb.status_host_cap < (size_t)n) {
    if (eb.status_host) {
      CQM_HIP(hipStreamSynchronize(s));
      CQM_HIP(hipHostFree(eb.status_host));
      CQM_HIP(hipHostFree(eb.status_norms));
    }
    eb.status_host = nullptr;
    eb.status_norms = nullptr;
    eb.status_host_cap = 0;
    const size_t c = std::max<size_t>((size_t)n, 256);  // systems
    CQM_HIP(hipHostMalloc((void**)&eb.status_host, sizeof(int) * kSysiStride * c, hipHostMallocDefault));
    CQM_HIP(hipHostGetDevicePointer((void**)&eb.status_host_dev, eb.status_host, 0));
    CQM_HIP(hipHostMalloc((void**)&eb.status_norms, sizeof(double) * 3 * c, hipHostMallocDefault));
    CQM_HIP(hipHostGetDevicePointer((void**)&eb.status_norms_dev, eb.status_norms, 0));
    eb.status_host_cap = c;
  }
  if (eb.cyc_cap < (size_t)n + 1) {
    if (eb.cyc_host) {
      CQM_HIP(hipStreamSynchronize(s));
      CQM_HIP(hipHostFree(eb.cyc_host));
    }
    eb.cyc_host = nullptr;
    eb.cyc_cap = 0;
    const size_t c = std::max<size_t>((size_t)n + 1, 256);
    CQM_HIP(hipHostMalloc((void**)&eb.cyc_host, sizeof(int) * c, hipHostMallocDefault));
    CQM_HIP(hipHostGetDevicePointer((void**)&eb.cyc_host_dev, eb.cyc_host, 0));
    eb.cyc_cap = c;
  }
  for (int k = 0; k < n; ++k) hd_[k].hflag = eb.cyc_host_dev + 1 + k;
  CQM_HIP(hipMemcpyAsync(eb.desc, hd_.data(), sizeof(SysDesc) * n, hipMemcpyHostToDevice, s));
  // graph-captured steps: every state in the stored form, no profiling
  bool eligible = !lite_.empty();
  for (SolveState* st : S_)
    eligible = eligible && dense_form(*st->p) && st->p->opt.graphs && !st->p->opt.profile;
  const bool same = prev_hd_.size() == hd_.size() && prev_split_ == split_ && prev_pre_ == anypre_ &&
                    std::memcmp(prev_hd_.data(), hd_.data(), sizeof(SysDesc) * hd_.size()) == 0;
  if (!eligible || !same) drop_graphs();
  graphs_ = eligible;
  prev_hd_ = hd_;
  prev_split_ = split_;
  prev_pre_ = anypre_;
  if (graphs_) {
    // the full group list, sorted by mesh size, in its own device buffer
    std::vector<int> ord(lite_.size());
    for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return lite_[a].M < lite_[b].M; });
    std::vector<GroupLite> all;
    all_cls_.clear();
    for (int gi : ord) {
      const GroupLite& g = lite_[gi];
      if (all_cls_.empty() || all_cls_.back().M != g.M)
        all_cls_.push_back(GClass{g.M, (int)all.size(), 0, false});
      all_cls_.back().count += 1;
      all_cls_.back().grouped |= g.n > 1;
      all.push_back(g);
    }
    const GroupLite* old_ptr = eb.all_groups;
    ensure(eb.all_groups, eb.all_cap, all.size());
    if (eb.all_groups != old_ptr) drop_graphs();
    CQM_HIP(hipMemcpyAsync(eb.all_groups, all.data(), sizeof(GroupLite) * all.size(),
                           hipMemcpyHostToDevice, s));
    if ((int)gexec_.size() != m_) {
      drop_graphs();
      gexec_.assign(m_, nullptr);
    }
  }
  flags_.assign((size_t)kSysiStride * n, 0);
}

void release_engine_bufs(EngineBufs& b) {
  if (b.desc) (void)hipFree(b.desc);
  if (b.groups) (void)hipFree(b.groups);
  if (b.status_host) (void)hipHostFree(b.status_host);
  if (b.cyc_host) (void)hipHostFree(b.cyc_host);
  if (b.status_norms) (void)hipHostFree(b.status_norms);
  if (b.open_cycle) (void)hipFree(b.open_cycle);
  if (b.open_step) (void)hipFree(b.open_step);
  if (b.staging) (void)hipHostFree(b.staging);
  if (b.all_groups) (void)hipFree(b.all_groups);
  b = EngineBufs{};
}

Engine::~Engine() {
  drop_graphs();
  if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
}

void Engine::drop_graphs() {
  for (hipGraphExec_t g : gexec_)
    if (g) (void)hipGraphExecDestroy(g);
  gexec_.clear();
}

// Spin on the progress word until the last kernel of step target - 1 has
// started; a wait beyond a few hundred milliseconds falls back to draining
// the stream (which also reports a device error).
void Engine::wait_progress(int target, hipStream_t s) {
  const volatile int* prog = eb.cyc_host;
  if (*prog >= target) return;
  const auto t0 = std::chrono::steady_clock::now();
  while (*prog < target) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(300)) {
      CQM_HIP(hipStreamSynchronize(s));
      return;
    }
    __builtin_ia32_pause();  // spin-wait hint to the core
  }
}

void Engine::init(int k, hipStream_t s) {
  SolveState* st = S_[k];
  Timed t(*S_[0]->p, CQM_K_OTHER, s);
  launch_gmres_init(eb.desc + st->first, st->p->Fsys, s);
}

void Engine::status(hipStream_t s) {
  const int n = (int)hd_.size();
  if (!n) return;
  // flags and norms of every system straight into pinned host memory
  launch_gather_diag(eb.desc, n, eb.status_host_dev, eb.status_norms_dev, s);
  CQM_HIP(hipStreamSynchronize(s));
  std::copy(eb.status_host, eb.status_host + flags_.size(), flags_.begin());
}

// Groups with a member whose flag `which` (0 system open, 1 cycle open) is
// set in the host copy of the flags, sorted by mesh size, uploaded through
// the pinned staging area.  The stream was synchronised by the status read,
// so the previous upload from the same staging area is complete.
void Engine::upload_arnoldi(int slot, hipStream_t s) {
  const int n = (int)hd_.size();
  SysDesc* st = eb.arn_staging + (size_t)slot * n;
  int c = 0;
  for (int k = 0; k < n; ++k)
    if (flags_[(size_t)kSysiStride * k + 1]) st[c++] = hd_[k];
  arn_n_ = c;
  if (c) CQM_HIP(hipMemcpyAsync(eb.arn_desc, st, sizeof(SysDesc) * c, hipMemcpyHostToDevice, s));
}

void Engine::upload_open(int which, GroupLite* dst, size_t stage, std::vector<GClass>& cls,
                         hipStream_t s) {
  cls.clear();
  if (lite_.empty()) return;
  std::vector<int> open;
  for (size_t gi = 0; gi < groups_.size(); ++gi) {
    bool any = false;
    for (int q = 0; q < groups_[gi].n; ++q)
      any |= flags_[(size_t)kSysiStride * groups_[gi].sys[q] + which] != 0;
    if (any) open.push_back((int)gi);
  }
  std::stable_sort(open.begin(), open.end(),
                   [&](int a, int b) { return lite_[a].M < lite_[b].M; });
  GroupLite* st = eb.staging + stage;
  for (size_t k = 0; k < open.size(); ++k) {
    const GroupLite& g = lite_[open[k]];
    st[k] = g;
    if (cls.empty() || cls.back().M != g.M) cls.push_back(GClass{g.M, (int)k, 0, false});
    cls.back().count += 1;
    cls.back().grouped |= g.n > 1;
  }
  if (!open.empty())
    CQM_HIP(hipMemcpyAsync(dst, st, sizeof(GroupLite) * open.size(), hipMemcpyHostToDevice, s));
}

template <typename R>
void Engine::dense_product(const GroupLite* list, const std::vector<GClass>& cls, int which, int j,
                           bool reduce, unsigned long long* ctr, hipStream_t s) {
  // preconditioned Arnoldi steps: P v_j waits in slot j + 1 for the product
  const int xj = which == 0 && pre_ ? j + 1 : j;
  for (const GClass& c : cls)
    launch_dense_gemv_groups<R>(list + c.off, c.count, c.M, c.grouped, which, xj, ctr, s);
  if (reduce && !cls.empty())
    launch_dense_reduce_desc<R>(eb.desc, (int)hd_.size(), maxM_, which, j, s);
}

bool Engine::state_done(int k) const {
  const SolveState* st = S_[k];
  for (int l = 0; l < st->p->Fsys; ++l)
    if (flags_[(size_t)kSysiStride * (st->first + l)]) return false;
  return true;
}

int Engine::cycle(hipStream_t s) { return mixed ? cycle_t<float>(s) : cycle_t<double>(s); }

// One restart cycle of every open system: start from the FP64 residual, up
// to m Arnoldi steps, update x, new FP64 residual.  Returns the number of
// systems that were open at the start (0: nothing was done).
// One Arnoldi step of every open system, launched directly: products of
// the stored-operator groups in `list` and of the other problems, then the
// Arnoldi kernels.
template <typename R>
void Engine::step_eager(int j, const GroupLite* list, const std::vector<GClass>& cls, hipStream_t s) {
  Problem& p0 = *S_[0]->p;
  const int n = (int)hd_.size();
  if (!lite_.empty()) {
    const int c = sizeof(R) == 4 ? CQM_K_GEMV32 : CQM_K_GEMV64;
    Timed t(p0, c, s);
    if (anypre_ && (j == 0 || !fuse_pre<R>())) launch_block_apply<R>(eb.desc, n, maxM_, j, s);
    dense_product<R>(list, cls, 0, j, !split_, p0.timer.ctr(c), s);
  } else if (anypre_ && (j == 0 || !fuse_pre<R>())) {
    launch_block_apply<R>(eb.desc, n, maxM_, j, s);
  }
  for (SolveState* st : S_) {
    Problem& p = *st->p;
    if (dense_form(p)) continue;
    const int M = (int)p.M;
    const int64_t bs = (int64_t)(m_ + 1) * M;
    cplx<R>* basis = reinterpret_cast<cplx<R>*>(st->base + st->basis);
    if (p.lay.pinv) {
      // preconditioned: the product of P v_j, formed in r's memory
      const cplx<R>* z = reinterpret_cast<const cplx<R>*>(st->base + st->r);
      apply_op<R>(p, 0, p.Fsys, z, (int64_t)M * (int64_t)(sizeof(cf64) / sizeof(cplx<R>)),
                  basis + (int64_t)(j + 1) * M, bs, st->at<int>(st->sysi) + 1, s);
    } else {
      apply_op<R>(p, 0, p.Fsys, basis + (int64_t)j * M, bs, basis + (int64_t)(j + 1) * M, bs,
                  st->at<int>(st->sysi) + 1, s);
    }
  }
  Timed t(p0, CQM_K_ARNOLDI, s);
  // the systems open when the list was built (the others issue no loads;
  // one closed since then leaves at its flag)
  const bool listed = arn_n_ > 0;
  launch_arnoldi<R>(listed ? eb.arn_desc : eb.desc, listed ? arn_n_ : n, maxM_, j, split_, split_,
                    fuse_pre<R>(), p0.timer.ctr(CQM_K_ARNOLDI), eb.cyc_host_dev, s);
}

// The same step from its captured graph (captured on first use).
template <typename R> void Engine::step_graph(int j, hipStream_t s) {
  if (!gexec_[j]) {
    // captured on a private stream (the caller's may be the null stream,
    // which cannot be captured); nothing executes during capture
    if (!cap_stream_) CQM_HIP(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    CQM_HIP(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
    if (anypre_ && (j == 0 || !fuse_pre<R>()))
      launch_block_apply<R>(eb.desc, (int)hd_.size(), maxM_, j, cap_stream_);
    dense_product<R>(eb.all_groups, all_cls_, 0, j, !split_, nullptr, cap_stream_);
    launch_arnoldi<R>(eb.desc, (int)hd_.size(), maxM_, j, split_, split_, fuse_pre<R>(), nullptr,
                      eb.cyc_host_dev, cap_stream_);
    const hipError_t ec = hipStreamEndCapture(cap_stream_, &g);
    CQM_HIP(ec);
    const hipError_t e = hipGraphInstantiate(&gexec_[j], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    CQM_HIP(e);
  }
  CQM_HIP(hipGraphLaunch(gexec_[j], s));
}

template <typename R> int Engine::cycle_t(hipStream_t s) {
  Stage stage(sizeof(R) == 4 ? "restart_cycle_fp32" : "restart_cycle_fp64");
  const int n = (int)hd_.size();
  if (!n) return 0;
  Problem& p0 = *S_[0]->p;
  const SysDesc* sd = eb.desc;
  const double outer_tol = p0.opt.outer_tol;
  const double inner_tol = sizeof(R) == 4 ? std::max(p0.opt.inner_tol, 2e-7) : p0.opt.inner_tol;
  auto count = [&](int which) {
    status(s);
    int c = 0;
    for (int k = 0; k < n; ++k) c += flags_[(size_t)kSysiStride * k + which] != 0;
    return c;
  };
  // compressed inner operator with plain residuals: each cycle gains about
  // the approximation error, so the inner target follows the last gain
  const double relax = mode_is_h2(p0.opt.mode) && p0.opt.refine_plain ? 0.1 : 0.0;
  {
    Timed t(p0, CQM_K_OTHER, s);
    launch_cycle_start<R>(sd, n, outer_tol, inner_tol, relax, s);
  }
  const int open = count(0);
  if (open == 0) return 0;
  // systems open now are the ones whose cycle runs (and whose residual is
  // formed at its end)
  upload_open(0, eb.open_cycle, 0, cyc_cls_, s);
  if (!graphs_) upload_arnoldi(0, s);
  // which closing-residual launches this cycle needs: each system's choice
  // (status flag 4, set by its cycle start) came with the status read
  bool any_dd = false, any_64 = false;
  for (int k = 0; k < n; ++k) {
    if (!flags_[(size_t)kSysiStride * k + 1]) continue;
    (flags_[(size_t)kSysiStride * k + 4] ? any_dd : any_64) = true;
  }
  const GroupLite* step_list = eb.open_cycle;
  step_cls_ = cyc_cls_;
  // host copies of the cycle-open flags: set here for the systems whose
  // cycle starts (the stream is idle after the status read), then written by
  // the device at every step
  eb.cyc_host[0] = 0;
  for (int k = 0; k < n; ++k) eb.cyc_host[1 + k] = flags_[(size_t)kSysiStride * k + 1] != 0;
  int listed = open, upload_j = 0;  // groups in step_list, and the step it was built at
  for (int j = 0; j < m_; ++j) {
    if (graphs_) step_graph<R>(j, s);
    else step_eager<R>(j, step_list, step_cls_, s);
    // the host queues at most kAhead steps beyond the last started one
    if (j >= kAhead) wait_progress(j - kAhead + 1, s);
    // a cycle flag only ever drops to 0, so the device's latest writes can
    // be read at any time: all 0 means the steps still queued do nothing
    const volatile int* cf = eb.cyc_host + 1;
    int c = 0;
    for (int k = 0; k < n; ++k) {
      const int f = cf[k];
      flags_[(size_t)kSysiStride * k + 1] = f;
      c += f != 0;
    }
    if (c == 0) break;
    // eager lists drop the groups closed since the list was built once a
    // quarter of them has closed; the staging copy of the previous list was
    // queued before step j - kAhead + 1, whose last kernel has started
    if (!graphs_ && j - kAhead > upload_j && 4 * c <= 3 * listed) {
      upload_open(1, eb.open_step, lite_.size(), step_cls_, s);
      upload_arnoldi(1, s);
      step_list = eb.open_step;
      listed = c;
      upload_j = j;
    }
  }
  {
    Timed t(p0, CQM_K_OTHER, s);
    // x += V y, or x += P (V y) for preconditioned systems
    launch_cycle_finish<R>(sd, n, maxM_, s);
  }
  if (!lite_.empty()) {
    // residuals of the systems that ran this cycle (the list from its start)
    Timed t(p0, CQM_K_GEMV64, s);
    // the residual that closes the cycle, per system in double-double or
    // FP64 as its cycle start chose (status flag 4); each launch takes its
    // own systems and the others leave at once
    if (any_dd) {
      for (const GClass& c : cyc_cls_)
        launch_resid_dd_groups(eb.open_cycle + c.off, c.count, c.M, c.grouped,
                               p0.timer.ctr(CQM_K_GEMV64), s);
      if (!cyc_cls_.empty()) launch_resid_dd_reduce(eb.desc, (int)hd_.size(), maxM_, s);
    }
    if (any_64)
      dense_product<double>(eb.open_cycle, cyc_cls_, 1, 0, true, p0.timer.ctr(CQM_K_GEMV64), s);
  }
  bool other_forms = false;  // stored-form residuals are complete already
  for (SolveState* st : S_) {
    Problem& p = *st->p;
    if (dense_form(p)) continue;
    other_forms = true;
    const int M = (int)p.M;
    if (mode_is_h2(p.opt.mode) && p.opt.refine_plain)
      apply_plain_free<double>(p, 0, p.Fsys, st->at<cf64>(st->x), M, st->at<cf64>(st->r), M,
                               st->at<int>(st->sysi), s);
    else
      apply_op<double>(p, 0, p.Fsys, st->at<cf64>(st->x), M, st->at<cf64>(st->r), M,
                       st->at<int>(st->sysi), s);
  }
  if (other_forms) {
    Timed t(p0, CQM_K_OTHER, s);
    launch_residual_combine(sd, n, s);
  }
  ++cycles_run;
  return open;
}
template void Engine::dense_product<float>(const GroupLite*, const std::vector<GClass>&, int, int,
                                           bool, unsigned long long*, hipStream_t);
template void Engine::dense_product<double>(const GroupLite*, const std::vector<GClass>&, int, int,
                                            bool, unsigned long long*, hipStream_t);
template void Engine::step_eager<float>(int, const GroupLite*, const std::vector<GClass>&, hipStream_t);
template void Engine::step_eager<double>(int, const GroupLite*, const std::vector<GClass>&, hipStream_t);
template void Engine::step_graph<float>(int, hipStream_t);
template void Engine::step_graph<double>(int, hipStream_t);
template int Engine::cycle_t<float>(hipStream_t);
template int Engine::cycle_t<double>(hipStream_t);

// Closing status pass for state k: residual norms refreshed by one more
// cycle start (systems still open keep their flags) and the diagnostics.
void Engine::finish_diag(int k, hipStream_t s, bool refresh) {
  SolveState* st = S_[k];
  Problem& p = *st->p;
  const double outer_tol = p.opt.outer_tol;
  if (refresh) {
    // residual norms of the last cycle, then the status of every system
    const SysDesc* sd = eb.desc + st->first;
    if (mixed) launch_cycle_start<float>(sd, p.Fsys, outer_tol, std::max(p.opt.inner_tol, 2e-7), 0.0, s);
    else launch_cycle_start<double>(sd, p.Fsys, outer_tol, p.opt.inner_tol, 0.0, s);
    status(s);
  }
  // else the status read that found every system closed is still current
  const int* fl = eb.status_host + (size_t)kSysiStride * st->first;
  const double* nm = eb.status_norms + (size_t)3 * st->first;
  cqm_diag& d = st->diag;
  d.cycles = cycles_run;
  d.total_iters = d.max_iters = 0;
  d.max_rel_residual = 0.0;
  int open = 0, nan = 0;
  for (int l = 0; l < p.Fsys; ++l) {
    const int* f = &fl[(size_t)kSysiStride * l];
    d.total_iters += f[3];
    d.max_iters = std::max(d.max_iters, f[3]);
    const double bn = nm[3 * l], rn = nm[3 * l + 1];
    if (bn > 0) d.max_rel_residual = std::max(d.max_rel_residual, rn / bn);
    open += f[0] != 0;
    nan += nm[3 * l + 2] != 0.0;
  }
  d.converged = nan ? -1 : (open == 0 ? 1 : 0);
}

// Full solves of a set of states; states with the same inner precision share
// the engine's launches.
void solve_states(std::vector<SolveState*>& S, hipStream_t s) {
  for (int g = 0; g < 2; ++g) {
    std::vector<SolveState*> G;
    for (SolveState* st : S)
      if ((mode_is_mixed(st->p->opt.mode) ? 1 : 0) == g) G.push_back(st);
    if (G.empty()) continue;
    Problem& p0 = *G[0]->p;
    p0.timer.on = p0.opt.profile != 0;
    p0.timer.reset(s);
    for (size_t k = 1; k < G.size(); ++k)
      if (G[k]->p != &p0) G[k]->p->timer.on = false;
    // what the shared launches need in common, checked before any work
    int pre = -1;
    for (SolveState* st : G) {
      const Problem& p = *st->p;
      require(p.opt.gmres_restart == p0.opt.gmres_restart, CQM_EINVAL,
              "batched problems must share gmres_restart");
      if (!dense_form(p)) continue;
      const int pk = p.lay.pinv != 0;
      require(pre < 0 || pk == pre, CQM_EINVAL,
              "batched stored-operator problems must share the preconditioner");
      pre = pk;
    }
    if (G.size() > 1) {
      // several problems: one work-queue launch assembles their stored
      // operators; the setup events of each bracket the whole batch setup
      for (SolveState* st : G)
        for (hipEvent_t& e : st->p->setup_ev)
          if (!e) CQM_HIP(hipEventCreate(&e));
      for (SolveState* st : G) CQM_HIP(hipEventRecord(st->p->setup_ev[0], s));
      prepare_batch(G, s);
      for (SolveState* st : G) CQM_HIP(hipEventRecord(st->p->setup_ev[1], s));
      for (SolveState* st : G) {
        pre_solve(*st, s, false);
        st->diag.t_setup_ms = -1.0;  // pending: read from the events after the solve
      }
    } else {
      for (SolveState* st : G) pre_solve(*st, s, true, true);
    }
    auto t1 = std::chrono::steady_clock::now();
    // a problem's own solve keeps its engine (buffers, captured graphs)
    std::unique_ptr<Engine> local;
    Engine* Ep;
    if (G.size() == 1 && G[0] == &p0.own) {
      if (!p0.engine) p0.engine = new Engine(*p0.ctx, p0.engine_bufs);
      Ep = p0.engine;
    } else {
      local = std::make_unique<Engine>(*p0.ctx);
      Ep = local.get();
    }
    Engine& E = *Ep;
    E.cycles_run = 0;
    E.set(G, s);
    for (size_t k = 0; k < G.size(); ++k) E.init((int)k, s);
    // a loop ended by convergence has just refreshed every residual norm
    bool converged = false;
    for (int c = 0; c < p0.opt.max_cycles && !converged; ++c) converged = E.cycle(s) == 0;
    for (size_t k = 0; k < G.size(); ++k) E.finish_diag((int)k, s, !converged);
    for (SolveState* st : G) post_solve(*st, s);
    const double el = ms_since(t1);
    if (p0.timer.on) p0.timer.collect(G[0]->diag.kernel_ms, G[0]->diag.kernel_calls, G[0]->diag.kernel_work);
    for (SolveState* st : G) {
      st->diag.t_solve_ms = el;
      st->p->last = st->diag;
    }
  }
}

}  // namespace cqm
