// Time-marching solve (Section 3.2, eq. dft, cqmgalapx, cqmrhs).  Stored
// plain form: the operator's distinct frequencies are transformed into the
// real integration weights What_n.  Compressed form (Section 6.2, eq.
// fastdft): the MACA fibres are transformed instead, so every weight is the
// compressed operator with transformed fibres.  Then step by step the
// history sum of eq. cqmrhs is formed on the device and What_0 q_n = r_n is
// solved by block-Jacobi preconditioned conjugate gradients (What_0 is real
// symmetric positive definite; the paper factorises it once, this build
// iterates on it).
#include <chrono>
#include <cmath>
#include <optional>

#include "internal.h"

namespace cqm {

void h2_stats(const Problem& p, cqm_diag* d);  // h2.cpp

namespace {
template <typename T> T* wsp(Problem& p, size_t off) { return reinterpret_cast<T*>(p.ws + off); }
double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}
}  // namespace

namespace {
// CG vectors and partials in the workspace region at lay.mvec
CgVec cg_vectors(Problem& p, const cf64* pinv) {
  const int M = (int)p.M;
  const int nwg = (M + 255) / 256;
  double* vb = wsp<double>(p, p.lay.mvec);
  CgVec v{};
  v.r = vb;
  v.z = vb + M;
  v.p = vb + 2 * (size_t)M;
  v.w = vb + 3 * (size_t)M;
  v.rz = vb + 5 * (size_t)M;  // [2][nwg]
  v.pw = v.rz + 2 * nwg;
  v.rr = v.pw + nwg;
  v.bb = v.rr + nwg;
  v.done = reinterpret_cast<int*>(v.bb + nwg);
  v.hdone = p.march_host;
  v.iters = p.march_host + 1;
  v.pinv = pinv;
  v.M = M;
  v.nwg = nwg;
  return v;
}

// Final relative residual of a step's CG from its partials (host sums).
double cg_residual(const CgVec& v, double* srr_out) {
  std::vector<double> rr(v.nwg), bb(v.nwg);
  CQM_HIP(hipMemcpy(rr.data(), v.rr, sizeof(double) * v.nwg, hipMemcpyDeviceToHost));
  CQM_HIP(hipMemcpy(bb.data(), v.bb, sizeof(double) * v.nwg, hipMemcpyDeviceToHost));
  double srr = 0.0, sbb = 0.0;
  for (int k = 0; k < v.nwg; ++k) srr += rr[k], sbb += bb[k];
  *srr_out = srr;
  return sbb > 0 ? std::sqrt(srr / sbb) : 0.0;
}

// Compressed operator: weights from the transformed fibres; the history sum
// and every CG product are compressed products (complex, real part kept:
// the transformed tensor is real up to its approximation error).
void solve_marching_h2(Problem& p, double* q_out, cqm_diag* diag, hipStream_t s) {
  require(p.full_band(), CQM_EINVAL,
          "compressed time marching needs the full band of frequencies (aca_band = CQM_BAND_FULL)");
  require(p.lay.mz != 0 && p.lay.diag64 != 0, CQM_EINVAL,
          "compressed time marching needs marching = 1 and the block-Jacobi preconditioner at "
          "problem creation (What_0's diagonal blocks come from the plain operator's)");
  const int M = (int)p.M, N = p.N;
  auto t0 = std::chrono::steady_clock::now();
  prepare_operator(p, s);  // MACA, near values, diagonal blocks of every frequency
  p.own.p = &p;
  p.own.base = p.ws;
  double* b = p.own.at<double>(p.own.b);
  cf64* dg = wsp<cf64>(p, p.lay.mdiag);
  cf64* pinv = wsp<cf64>(p, p.lay.mpinv);
  {
    Stage setup("marching_weights");
    launch_rhs(p, p.inc, b, s);
    h2_marching_weights(p, s);
    launch_freq_mean_blocks(wsp<cf64>(p, p.lay.diag64), p.Fsys, block_inverse_elems(M), dg, s);
    launch_block_inverse<double>(dg, M, 1, true, pinv, s);
    CQM_HIP(hipStreamSynchronize(s));
  }
  const double t_setup = ms_since(t0);
  auto t1 = std::chrono::steady_clock::now();
  CgVec v = cg_vectors(p, pinv);
  cf64* HX = wsp<cf64>(p, p.lay.mz);  // row m: q_m as complex, cluster order
  cf64* Y = wsp<cf64>(p, p.lay.my);   // the history sum of the current step
  cf64* pc = wsp<cf64>(p, p.lay.mpc);
  cf64* wc = pc + M;
  // the weights carry the compressed operator's approximation error, far
  // above 1e-12; a tighter CG gains nothing
  const double tol = std::max(p.opt.outer_tol, 1e-12);
  const double tol2 = tol * tol;
  constexpr int kMaxIter = 500, kCheck = 2;
  int total = 0, worst = 0;
  bool converged = true, finite = true;
  double max_res = 0.0;
  Stage steps("marching_steps");
  for (int n = 0; n <= N; ++n) {
    if (n == 0) {
      CQM_HIP(hipMemcpyAsync(v.r, b, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    } else {
      // sum_{k=1}^{n} What_k q_{n-k} by the fast right-hand side (eq. fastrhs)
      h2_history_sum(p, n, HX, Y, s);
      launch_hist_reduce(Y, 1, M, b + (size_t)n * M, v.r, s);
    }
    v.x = q_out + (size_t)n * M;
    p.march_host[0] = 0;
    launch_cg_init(v, s);
    for (int it = 0; it < kMaxIter; ++it) {
      launch_cg_check(v, tol2, s);
      launch_to_complex(v.p, M, pc, v.done, s);
      h2_apply_weights(p, 0, 1, pc, M, wc, M, s);
      launch_cg_reduce_complex(v, wc, s);
      launch_cg_finish(v, it & 1, s);
      if ((it + 1) % kCheck == 0) {
        CQM_HIP(hipStreamSynchronize(s));
        if (*(volatile int*)&p.march_host[0]) break;
      }
    }
    CQM_HIP(hipStreamSynchronize(s));
    const int it = *(volatile int*)&p.march_host[1];
    total += it;
    worst = std::max(worst, it);
    double srr = 0.0;
    const double res = cg_residual(v, &srr);
    if (!std::isfinite(res)) finite = false;
    if (!(res <= tol) && !(srr == 0.0)) converged = false;
    max_res = std::max(max_res, res);
    if (n < N) {
      launch_to_complex(v.x, M, pc, nullptr, s);
      h2_history_push(p, n, pc, HX + (size_t)n * M, s);
    }
  }
  cqm_diag d{};
  d.n_systems = N + 1;
  d.total_iters = total;
  d.max_iters = worst;
  d.max_rel_residual = finite ? max_res : NAN;
  d.t_setup_ms = t_setup;
  d.t_solve_ms = ms_since(t1);
  d.converged = converged && finite ? 1 : 0;
  h2_stats(p, &d);
  p.last = d;
  if (diag) *diag = d;
  if (!finite) throw Error(CQM_ENAN, "non-finite residual in the marching solve");
  if (!converged) throw Error(CQM_ENOCONV, "a marching step missed its tolerance");
}
}  // namespace

void solve_marching(Problem& p, double* q_out, cqm_diag* diag, hipStream_t s) {
  require(p.opt.formulation == CQM_FORMULATION_INDIRECT, CQM_EINVAL,
          "the marching solve takes the indirect formulation");
  require(p.opt.marching != 0, CQM_EINVAL,
          "create the problem with cqm_options.marching = 1 (the workspace holds the weights)");
  require(p.ws != nullptr && p.ws_bytes >= p.lay.total, CQM_ENOMEM, "workspace missing");
  require(q_out != nullptr, CQM_EINVAL, "NULL output");
  require(p.inc.kind != 0, CQM_EINVAL, "no incident data (cqm_set_plane_wave or samples)");
  CQM_HIP(hipSetDevice(p.ctx->device));
  if (!p.march_host) {
    CQM_HIP(hipHostMalloc((void**)&p.march_host, sizeof(int) * 4, hipHostMallocDefault));
    p.march_host[0] = p.march_host[1] = 0;
  }
  if (mode_is_h2(p.opt.mode)) {
    solve_marching_h2(p, q_out, diag, s);
    return;
  }
  require(p.opt.form == CQM_FORM_DENSE && p.lay.mw != 0, CQM_EINVAL,
          "time marching needs the stored form (CQM_FORM_DENSE) or a compressed mode");
  const int M = (int)p.M, F = p.F, N = p.N;
  auto t0 = std::chrono::steady_clock::now();
  // operator (near field, FP64 assembly), right-hand sides b_n
  prepare_operator(p, s);
  std::optional<Stage> setup;
  setup.emplace("marching_weights");
  SolveState& st = p.own;
  st.p = &p;
  st.base = p.ws;
  double* b = st.at<double>(st.b);
  launch_rhs(p, p.inc, b, s);
  // weights What_n and the block inverses of What_0
  double* W = wsp<double>(p, p.lay.mw);
  cf64* dg = wsp<cf64>(p, p.lay.mdiag);
  cf64* pinv = wsp<cf64>(p, p.lay.mpinv);
  launch_march_weights(wsp<cf64>(p, p.lay.dense64), M, p.Fh, F, p.dev.tw_inv, p.dev.rho_ipow, W, s);
  launch_march_diag(W, M, dg, s);
  launch_block_inverse<double>(dg, M, 1, true, pinv, s);
  CQM_HIP(hipStreamSynchronize(s));
  setup.reset();
  const double t_setup = ms_since(t0);
  auto t1 = std::chrono::steady_clock::now();
  CgVec v = cg_vectors(p, pinv);
  double* P = wsp<double>(p, p.lay.mpart);
  const double tol = p.opt.outer_tol > 0 ? std::max(p.opt.outer_tol, 1e-16) : 1e-15;
  const double tol2 = tol * tol;
  constexpr int kMaxIter = 500;
  int total = 0, worst = 0, last = 8;
  bool converged = true, finite = true;
  double max_res = 0.0;
  Stage steps("marching_steps");
  for (int n = 0; n <= N; ++n) {
    // r_n = b_n - sum_{j=1}^{n} What_j q_{n-j}
    if (n == 0) {
      CQM_HIP(hipMemcpyAsync(v.r, b, sizeof(double) * M, hipMemcpyDeviceToDevice, s));
    } else {
      const int S = march_chunks(M, n);
      launch_march_product(W, M, 1, n, q_out, n - 1, P, S, nullptr, s);
      launch_march_reduce(P, S, M, -1.0, b + (size_t)n * M, v.r, s);
    }
    // What_0 q_n = r_n, q_n written in place (row n of q)
    v.x = q_out + (size_t)n * M;
    p.march_host[0] = 0;
    launch_cg_init(v, s);
    int issued = 0, batch = last;
    for (;;) {
      for (int k = 0; k < batch; ++k, ++issued) launch_cg_iteration(v, W, P, issued & 1, tol2, s);
      CQM_HIP(hipStreamSynchronize(s));
      if (*(volatile int*)&p.march_host[0] || issued >= kMaxIter) break;
      batch = 2;
    }
    const int it = *(volatile int*)&p.march_host[1];
    last = std::max(1, it);
    total += it;
    worst = std::max(worst, it);
    double srr = 0.0;
    const double res = cg_residual(v, &srr);
    if (!std::isfinite(res)) finite = false;
    if (!(res <= tol) && !(srr == 0.0)) converged = false;
    max_res = std::max(max_res, res);
  }
  cqm_diag d{};
  d.n_systems = N + 1;
  d.total_iters = total;
  d.max_iters = worst;
  d.max_rel_residual = finite ? max_res : NAN;
  d.t_setup_ms = t_setup;
  d.t_solve_ms = ms_since(t1);
  d.operator_bytes = (int64_t)(sizeof(double) * (size_t)F * sym_slice(M));
  d.converged = converged && finite ? 1 : 0;
  p.last = d;
  if (diag) *diag = d;
  if (!finite) throw Error(CQM_ENAN, "non-finite residual in the marching solve");
  if (!converged) throw Error(CQM_ENOCONV, "a marching step missed its tolerance");
}

}  // namespace cqm
