// extern "C" entry points and the solve driver of the plain operator forms.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

namespace cqm {
void h2_release(Problem& p);                 // h2.cpp
void h2_stats(const Problem& p, cqm_diag* d);
}  // namespace cqm

namespace cqm {
void KernelTimer::begin(int c, hipStream_t s) {
  if (!on) return;
  while (pool.size() < used + 2) {
    hipEvent_t e;
    CQM_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  cls.push_back(c);
  CQM_HIP(hipEventRecord(pool[used], s));
}
void KernelTimer::end(hipStream_t s) {
  if (!on) return;
  if (hipEventRecord(pool[used + 1], s) == hipSuccess) used += 2;
}
void KernelTimer::reset(hipStream_t s) {
  cls.clear();
  used = 0;
  if (!on) return;
  if (!work_d) CQM_HIP(hipMalloc(&work_d, sizeof(unsigned long long) * CQM_K_CLASSES));
  CQM_HIP(hipMemsetAsync(work_d, 0, sizeof(unsigned long long) * CQM_K_CLASSES, s));
}
void KernelTimer::collect(double* ms, int* calls, double* work) {
  if (work_d && work) {
    unsigned long long w[CQM_K_CLASSES];
    CQM_HIP(hipMemcpy(w, work_d, sizeof(w), hipMemcpyDeviceToHost));
    for (int c = 0; c < CQM_K_CLASSES; ++c) work[c] += (double)w[c];
  }
  for (size_t k = 0; k < cls.size() && 2 * k + 1 < used + 1 && 2 * k + 1 < pool.size(); ++k) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess) {
      ms[cls[k]] += t;
      calls[cls[k]] += 1;
    }
  }
  cls.clear();
  used = 0;
}
void KernelTimer::release() {
  if (work_d) (void)hipFree(work_d);
  work_d = nullptr;
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
  cls.clear();
  used = 0;
}
}  // namespace cqm

using namespace cqm;


namespace {
thread_local std::string g_last_error = "no error";

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
}  // namespace

int cqm::fail_with(int code, const std::string& msg) { return fail(code, msg); }

namespace {

template <typename F> int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(CQM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(CQM_EINVAL, e.what());
  }
}

void frequencies_host(int N, double T, double rho, std::vector<double>& re, std::vector<double>& im,
                      double& rho_out) {
  const int F = N + 1;
  const double dt = T / N;
  if (rho <= 0.0) rho = std::pow(10.0, -8.0 / N);
  rho_out = rho;
  re.resize(F);
  im.resize(F);
  for (int l = 0; l < F; ++l) {
    // xi = rho zeta^-l, s = (3/2 - 2 xi + xi^2/2)/dt  (BDF2)
    const double c = std::cos(2.0 * M_PI * l / F), sn = -std::sin(2.0 * M_PI * l / F);
    const double xr = rho * c, xi = rho * sn;
    const double x2r = xr * xr - xi * xi, x2i = 2.0 * xr * xi;
    re[l] = (1.5 - 2.0 * xr + 0.5 * x2r) / dt;
    im[l] = (-2.0 * xi + 0.5 * x2i) / dt;
  }
}

int finish(int rc) {
  if (rc == CQM_ENAN) return fail(rc, "non-finite residual in some frequency system");
  if (rc == CQM_ENOCONV) return fail(rc, "some frequency systems missed outer_tol");
  return rc;
}
}  // namespace

extern "C" {

const char* cqm_last_error(void) { return g_last_error.c_str(); }

int cqm_default_options(cqm_options* o) {
  if (!o) return fail(CQM_EINVAL, "options pointer is NULL");
  std::memset(o, 0, sizeof(*o));
  o->mode = CQM_MIXED_PLAIN;
  o->form = CQM_FORM_DENSE;
  o->rho = 0.0;
  o->gmres_restart = 30;
  o->max_cycles = 60;
  o->inner_tol = 1e-8;
  o->outer_tol = 1e-15;
  o->n_min = 32;
  o->eta = 1.0;
  o->cheb_m = 4;
  o->eps_aca = 1e-6;
  o->aca_band = CQM_BAND_FULL;
  o->q_duffy = 5;
  o->reuse_operator = 0;
  o->autotune = 1;
  o->graphs = 0;
  o->precond = CQM_PRECOND_BLOCK_JACOBI;
  o->cutoff_inner = 18.0;
  o->cutoff_outer = 45.0;
  o->refine_plain = 1;
  o->formulation = CQM_FORMULATION_INDIRECT;
  return CQM_OK;
}

int cqm_ctx_create(int device, cqm_ctx_t* out) {
  return guarded([&] {
    require(out != nullptr, CQM_EINVAL, "out is NULL");
    int n = 0;
    CQM_HIP(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, CQM_EINVAL, "device index out of range");
    CQM_HIP(hipSetDevice(device));
    far_scratch_init(device);  // device address of the fixed scratch array, once per device
    auto* c = new cqm_ctx_s();
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        cus > 0)
      c->cus = cus;
    *out = c;
    return CQM_OK;
  });
}

int cqm_ctx_destroy(cqm_ctx_t ctx) {
  if (!ctx) return CQM_OK;
  (void)hipSetDevice(ctx->device);
  release_engine_bufs(ctx->eb);
  if (ctx->asm_jobs) (void)hipFree(ctx->asm_jobs);
  if (ctx->asm_stage) (void)hipHostFree(ctx->asm_stage);
  if (ctx->asm_counter) (void)hipFree(ctx->asm_counter);
  delete ctx;
  return CQM_OK;
}

int cqm_problem_create(cqm_ctx_t ctx, const double* vertices, int64_t nv, const int32_t* tris,
                       int64_t M, int32_t N, double T, const cqm_options* opt,
                       cqm_problem_t* out) {
  return guarded([&] {
    require(ctx && vertices && tris && out, CQM_EINVAL, "NULL argument");
    require(nv >= 3 && M >= 1 && M < (1 << 30), CQM_EINVAL, "bad mesh sizes");
    require(N >= 2 && N <= 4096, CQM_EINVAL, "N must be in [2, 4096]");
    require(T > 0 && std::isfinite(T), CQM_EINVAL, "T must be positive");
    cqm_options o;
    cqm_default_options(&o);
    if (opt) o = *opt;
    require(o.mode >= 0 && o.mode <= 3, CQM_EINVAL, "unknown mode");
    require(o.form == CQM_FORM_DENSE || o.form == CQM_FORM_MATRIX_FREE, CQM_EINVAL, "unknown form");
    require(o.gmres_restart >= 2 && o.gmres_restart <= 64, CQM_EINVAL, "gmres_restart in [2,64]");
    require(o.max_cycles >= 1, CQM_EINVAL, "max_cycles >= 1");
    require(o.q_duffy >= 1 && o.q_duffy <= kMaxDuffy, CQM_EINVAL, "q_duffy in [1,16]");
    require(o.inner_tol > 0 && o.outer_tol >= 0, CQM_EINVAL, "tolerances");
    require(o.rho >= 0 && o.rho < 1, CQM_EINVAL, "rho in [0,1)");
    require(o.cheb_m >= 2 && o.cheb_m <= 8, CQM_EINVAL, "cheb_m in [2,8]");
    require(o.n_min >= 2 && o.eta > 0 && o.eps_aca > 0, CQM_EINVAL, "tree / ACA parameters");
    require(o.aca_band == CQM_BAND_FULL || o.aca_band == CQM_BAND_HALF, CQM_EINVAL, "aca_band");
    require(o.arnoldi_layout >= CQM_ARNOLDI_AUTO && o.arnoldi_layout <= CQM_ARNOLDI_SPLIT, CQM_EINVAL,
            "arnoldi_layout");
    require(o.precond == CQM_PRECOND_NONE || o.precond == CQM_PRECOND_BLOCK_JACOBI, CQM_EINVAL,
            "precond");
    require(o.cutoff_inner >= 0 && o.cutoff_outer >= 0 && std::isfinite(o.cutoff_inner) &&
                std::isfinite(o.cutoff_outer),
            CQM_EINVAL, "cut-off exponents must be finite and >= 0");
    require(o.formulation == CQM_FORMULATION_INDIRECT || o.formulation == CQM_FORMULATION_DIRECT,
            CQM_EINVAL, "unknown formulation");
    for (int64_t k = 0; k < 3 * nv; ++k)
      require(std::isfinite(vertices[k]), CQM_EINVAL, "non-finite vertex coordinate");
    for (int64_t k = 0; k < 3 * M; ++k)
      require(tris[k] >= 0 && tris[k] < nv, CQM_EINVAL, "triangle index out of range");
    CQM_HIP(hipSetDevice(ctx->device));
    auto* p = new cqm_problem_s();
    try {
      p->ctx = ctx;
      p->M = M;
      p->nv = nv;
      p->N = N;
      p->T = T;
      p->dt = T / N;
      p->F = N + 1;
      p->Fh = p->F / 2 + 1;
      p->opt = o;
      p->Fsys = (mode_is_h2(o.mode) && o.aca_band == CQM_BAND_FULL) ? p->F : p->Fh;
      p->verts.assign(vertices, vertices + 3 * nv);
      p->tris.assign(tris, tris + 3 * M);
      // degenerate triangles
      for (int64_t i = 0; i < M; ++i) {
        const double* A = &p->verts[3 * tris[3 * i]];
        const double* B = &p->verts[3 * tris[3 * i + 1]];
        const double* C = &p->verts[3 * tris[3 * i + 2]];
        double u[3], v[3], e = 0;
        for (int d = 0; d < 3; ++d) u[d] = B[d] - A[d], v[d] = C[d] - A[d], e = std::max(e, std::fabs(u[d]) + std::fabs(v[d]));
        const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        require(std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-12 * e * e, CQM_EINVAL,
                "degenerate triangle " + std::to_string(i));
      }
      frequencies_host(N, T, o.rho, p->s_re, p->s_im, p->rho);
      build_near(*p);
      upload_problem(*p);
      compute_layout(*p);
      const int64_t nnz = (int64_t)p->col.size();
      p->far_units = ((int64_t)M * M - nnz) * 36 * (int64_t)p->Fsys;
    } catch (...) {
      cqm_problem_destroy(p);
      throw;
    }
    *out = p;
    return CQM_OK;
  });
}

int cqm_problem_destroy(cqm_problem_t p) {
  if (!p) return CQM_OK;
  (void)hipSetDevice(p->ctx ? p->ctx->device : 0);
  h2_release(*p);
  p->timer.release();
  if (p->march_host) (void)hipHostFree(p->march_host);
  for (hipEvent_t e : p->setup_ev)
    if (e) (void)hipEventDestroy(e);
  delete p->engine;
  p->engine = nullptr;
  release_engine_bufs(p->engine_bufs);
  void* bufs[] = {p->dev.pts64, p->dev.pts32, p->dev.vid, p->dev.area, p->dev.verts,
                  p->dev.near_rowptr, p->dev.near_col, p->dev.near_row, p->dev.near_kind, p->dev.near_vtx,
                  p->dev.near_static, p->dev.gl, p->dev.s, p->dev.tw_fwd, p->dev.tw_inv,
                  p->dev.rho_pow, p->dev.rho_ipow, p->dev.ea64, p->dev.pb64, p->dev.ea64u, p->dev.pb64u, p->dev.ftab, p->dev.ea32,
                  p->dev.pb32, p->dev.tile_gap, p->dev.sub_box, p->dev.nrm64, p->dev.nearK_static, p->dev.near_tpos,
                  p->dev.nearD_static, p->dev.v2t_ptr, p->dev.v2t};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete p;
  return CQM_OK;
}

int cqm_workspace_size(cqm_problem_t p, size_t* bytes) {
  return guarded([&] {
    require(p && bytes, CQM_EINVAL, "NULL argument");
    *bytes = p->lay.total;
    return CQM_OK;
  });
}

int cqm_set_workspace(cqm_problem_t p, void* dev_ptr, size_t bytes) {
  return guarded([&] {
    require(p != nullptr, CQM_EINVAL, "NULL problem");
    require(dev_ptr != nullptr, CQM_EINVAL, "NULL workspace");
    require(((uintptr_t)dev_ptr & 255) == 0, CQM_EINVAL, "workspace must be 256-byte aligned");
    require(bytes >= p->lay.total, CQM_ENOMEM,
            "workspace too small: need " + std::to_string(p->lay.total) + " bytes");
    if ((char*)dev_ptr != p->ws) {
      p->near_ready = false;
      p->dense_ready = false;
    }
    p->ws = (char*)dev_ptr;
    p->ws_bytes = bytes;
    p->own.p = p;
    p->own.base = p->ws;
    return CQM_OK;
  });
}

int cqm_set_plane_wave(cqm_problem_t p, const double d[3], double sigma, double t0, double amp) {
  return guarded([&] {
    require(p && d, CQM_EINVAL, "NULL argument");
    const double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    require(n > 0 && std::isfinite(n), CQM_EINVAL, "direction must be a nonzero finite vector");
    require(sigma > 0 && std::isfinite(sigma) && std::isfinite(t0), CQM_EINVAL, "sigma/t0");
    require(std::isfinite(amp), CQM_ENAN, "non-finite amplitude");
    for (int k = 0; k < 3; ++k) p->inc.dir[k] = d[k] / n;
    p->inc.sigma = sigma;
    p->inc.t0 = t0;
    p->inc.amp = amp;
    p->inc.kind = 1;
    return CQM_OK;
  });
}

int cqm_set_dirichlet_samples(cqm_problem_t p, const double* g) {
  return guarded([&] {
    require(p && g, CQM_EINVAL, "NULL argument");
    p->inc.samples = g;
    p->inc.kind = 2;
    return CQM_OK;
  });
}

int cqm_solve(cqm_problem_t p, double* q_out, cqm_diag* diag, hipStream_t stream) {
  return guarded([&] {
    Stage stage("cqm_solve");
    require(p != nullptr, CQM_EINVAL, "NULL problem");
    p->own.p = p;
    p->own.base = p->ws;
    p->own.inc = p->inc;
    p->own.q_out = q_out;
    std::vector<SolveState*> S{&p->own};
    solve_states(S, stream);
    if (diag) *diag = p->own.diag;
    return finish(diag_status(p->own.diag));
  });
}

int cqm_solve_batch(cqm_problem_t* probs, int32_t count, double** q_outs, cqm_diag* diags,
                    hipStream_t stream) {
  return guarded([&] {
    Stage stage("cqm_solve_batch");
    require(probs && q_outs && count >= 0, CQM_EINVAL, "NULL argument");
    std::vector<SolveState*> S;
    for (int k = 0; k < count; ++k) {
      require(probs[k] != nullptr, CQM_EINVAL, "NULL problem in batch");
      for (int j = 0; j < k; ++j)
        require(probs[j] != probs[k], CQM_EINVAL, "a problem appears twice in the batch");
      Problem& p = *probs[k];
      p.own.p = &p;
      p.own.base = p.ws;
      p.own.inc = p.inc;
      p.own.q_out = q_outs[k];
      S.push_back(&p.own);
    }
    solve_states(S, stream);
    int worst = CQM_OK;
    for (int k = 0; k < count; ++k) {
      if (diags) diags[k] = probs[k]->own.diag;
      const int rc = diag_status(probs[k]->own.diag);
      if (rc != CQM_OK && (worst == CQM_OK || rc < worst)) worst = rc;
    }
    return finish(worst);
  });
}

int cqm_solve_marching(cqm_problem_t p, double* q_out, cqm_diag* diag, hipStream_t stream) {
  return guarded([&] {
    Stage stage("cqm_solve_marching");
    require(p != nullptr, CQM_EINVAL, "NULL problem");
    solve_marching(*p, q_out, diag, stream);
    return CQM_OK;
  });
}

int cqm_frequencies(int32_t N, double T, double rho, double* s_re, double* s_im) {
  return guarded([&] {
    require(N >= 1 && T > 0 && s_re && s_im && rho >= 0 && rho < 1, CQM_EINVAL, "bad arguments");
    std::vector<double> re, im;
    double r;
    frequencies_host(N, T, rho, re, im, r);
    std::copy(re.begin(), re.end(), s_re);
    std::copy(im.begin(), im.end(), s_im);
    return CQM_OK;
  });
}

int cqm_apply_V(cqm_problem_t p, int32_t l0, int32_t nl, int32_t precision, const void* x, void* y,
                hipStream_t stream) {
  return guarded([&] {
    require(p && x && y, CQM_EINVAL, "NULL argument");
    require(l0 >= 0 && nl >= 1 && l0 + nl <= p->Fsys, CQM_EINVAL, "frequency range outside the solved band");
    require(precision == 32 || precision == 64, CQM_EINVAL, "precision must be 32 or 64");
    CQM_HIP(hipSetDevice(p->ctx->device));
    require(p->ws != nullptr && p->ws_bytes >= p->lay.total, CQM_ENOMEM, "workspace missing");
    const bool reuse = p->opt.reuse_operator;
    p->opt.reuse_operator = 1;  // assemble once, then reuse across probes
    try {
      prepare_operator(*p, stream);
    } catch (...) {
      p->opt.reuse_operator = reuse;
      throw;
    }
    p->opt.reuse_operator = reuse;
    const int M = (int)p->M;
    if (precision == 32)
      apply_op<float>(*p, l0, nl, (const cf32*)x, M, (cf32*)y, M, nullptr, stream);
    else
      apply_op<double>(*p, l0, nl, (const cf64*)x, M, (cf64*)y, M, nullptr, stream);
    return CQM_OK;
  });
}

int cqm_apply_K(cqm_problem_t p, int32_t l0, int32_t nl, int32_t adjoint, const void* x, void* y,
                hipStream_t stream) {
  return guarded([&] {
    require(p && x && y, CQM_EINVAL, "NULL argument");
    require(p->opt.formulation == CQM_FORMULATION_DIRECT, CQM_EINVAL,
            "create the problem with formulation = CQM_FORMULATION_DIRECT");
    require(l0 >= 0 && nl >= 1 && l0 + nl <= p->Fsys, CQM_EINVAL, "frequency range outside the solved band");
    require(p->ws != nullptr && p->ws_bytes >= p->lay.total, CQM_ENOMEM, "workspace missing");
    CQM_HIP(hipSetDevice(p->ctx->device));
    prepare_double_layer(*p, stream);
    const int M = (int)p->M;
    launch_apply_K(*p, l0, nl, (const cf64*)x, M, nullptr, 0.0, (cf64*)y, M,
                   reinterpret_cast<const cf64*>(p->ws + p->lay.nearK),
                   reinterpret_cast<cf64*>(p->ws + p->lay.kpart), adjoint != 0, stream);
    return CQM_OK;
  });
}

int cqm_apply_D(cqm_problem_t p, int32_t l0, int32_t nl, const void* x, void* y, hipStream_t stream) {
  return guarded([&] {
    require(p && x && y, CQM_EINVAL, "NULL argument");
    require(p->opt.formulation == CQM_FORMULATION_DIRECT, CQM_EINVAL,
            "create the problem with formulation = CQM_FORMULATION_DIRECT");
    require(l0 >= 0 && nl >= 1 && l0 + nl <= p->Fsys, CQM_EINVAL, "frequency range outside the solved band");
    require(p->ws != nullptr && p->ws_bytes >= p->lay.total, CQM_ENOMEM, "workspace missing");
    CQM_HIP(hipSetDevice(p->ctx->device));
    // static parts, once per mesh: the single layer's (curl term) and the
    // weighted ones (s^2 term)
    if (!p->static_ready) {
      launch_near_static(*p, stream);
      p->static_ready = true;
    }
    if (!p->nearD_static_ready) {
      launch_nearD_static(*p, stream);
      p->nearD_static_ready = true;
    }
    launch_apply_D(*p, l0, nl, (const cf64*)x, p->nv, (cf64*)y, p->nv,
                   reinterpret_cast<cf64*>(p->ws + p->lay.dsrc),
                   reinterpret_cast<cf64*>(p->ws + p->lay.dpart),
                   reinterpret_cast<cf64*>(p->ws + p->lay.dz), stream);
    return CQM_OK;
  });
}

int cqm_apply_V_noalloc(cqm_problem_t p, int32_t l0, int32_t nl, int32_t precision, const void* x,
                        void* y, hipStream_t stream) {
  return guarded([&] {
    require(p && x && y, CQM_EINVAL, "NULL argument");
    require(!mode_is_h2(p->opt.mode) && p->opt.form == CQM_FORM_MATRIX_FREE, CQM_EINVAL,
            "the allocation-free product is for the matrix-free plain form");
    require(l0 >= 0 && nl >= 1 && l0 + nl <= p->Fsys, CQM_EINVAL, "frequency range outside the solved band");
    require(precision == 32 || precision == 64, CQM_EINVAL, "precision must be 32 or 64");
    const size_t slot = (size_t)nl * p->M * (precision == 32 ? sizeof(cf32) : sizeof(cf64));
    require(slot <= kFarScratchBytes, CQM_ENOMEM,
            "nl x M x element size = " + std::to_string(slot) + " bytes exceeds the fixed scratch of " +
                std::to_string(kFarScratchBytes) + " bytes");
    require(p->ws != nullptr && p->ws_bytes >= p->lay.total, CQM_ENOMEM, "workspace missing");
    CQM_HIP(hipSetDevice(p->ctx->device));
    // near-field values into the caller's workspace (launches only)
    if (!p->static_ready) {
      launch_near_static(*p, stream);
      p->static_ready = true;
    }
    cf64* nv = reinterpret_cast<cf64*>(p->ws + p->lay.near_val);
    if (!p->near_ready) {
      launch_near_values(*p, nv, stream);
      p->near_ready = true;
    }
    const int M = (int)p->M;
    if (precision == 32)
      launch_far_apply_fixed<float>(*p, l0, nl, (const cf32*)x, M, (cf32*)y, M, nv, stream);
    else
      launch_far_apply_fixed<double>(*p, l0, nl, (const cf64*)x, M, (cf64*)y, M, nv, stream);
    return CQM_OK;
  });
}

int cqm_near_entries(cqm_problem_t p, int64_t* nnz, int32_t* row_ptr, int32_t* col,
                     double* static_vals) {
  return guarded([&] {
    require(p && nnz, CQM_EINVAL, "NULL argument");
    *nnz = (int64_t)p->col.size();
    if (row_ptr) std::copy(p->rowptr.begin(), p->rowptr.end(), row_ptr);
    if (col) std::copy(p->col.begin(), p->col.end(), col);
    if (static_vals) {
      CQM_HIP(hipSetDevice(p->ctx->device));
      if (!p->static_ready) {
        launch_near_static(*p, nullptr);
        CQM_HIP(hipDeviceSynchronize());
        p->static_ready = true;
      }
      CQM_HIP(hipMemcpy(static_vals, p->dev.near_static, sizeof(double) * p->col.size(),
                        hipMemcpyDeviceToHost));
    }
    return CQM_OK;
  });
}

int cqm_operator_stats(cqm_problem_t p, cqm_diag* out) {
  return guarded([&] {
    require(p && out, CQM_EINVAL, "NULL argument");
    *out = p->last;
    out->far_units = p->far_units;
    out->n_systems = p->Fsys;
    if (mode_is_h2(p->opt.mode)) h2_stats(*p, out);
    return CQM_OK;
  });
}

}  // extern "C"
