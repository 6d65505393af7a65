// Internal declarations of the CQM-BEM library (host planner + HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cqm.h"

namespace cqm {

// ------------------------------------------------------------ errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define CQM_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      throw ::cqm::Error(CQM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline void require(bool ok, int code, const std::string& msg) {
  if (!ok) throw Error(code, msg);
}

// ------------------------------------------------------------ complex storage
struct __align__(8) cf32 {
  float re, im;
};
struct __align__(16) cf64 {
  double re, im;
};
template <typename R> struct CplxOf;
template <> struct CplxOf<float> { using T = cf32; };
template <> struct CplxOf<double> { using T = cf64; };
template <typename R> using cplx = typename CplxOf<R>::T;

// Quadrature point (x, y, z, weight*area) in a given precision.
template <typename R> struct Pt4;
template <> struct Pt4<float> { using T = float4; };
template <> struct Pt4<double> { using T = double4; };

constexpr int kQ = 6;          // Dunavant points per triangle
constexpr int kMaxDuffy = 16;  // max Gauss points per Duffy dimension
constexpr int kSysiStride = 4; // ints per system in the GMRES status array

// Per-frequency constants of the factor exp(-s r) = 2^(ea r) e^{-2 pi i pb r}:
// ea = -Re(s) log2(e), pb = Im(s) / (2 pi).  Padded with zero-work entries.
template <typename R> struct FreqTab {
  const R* ea;
  const R* pb;
};

// ------------------------------------------------------------ problem state
struct Ctx {
  int device = 0;
};

// Device tables of one mesh (owned by the problem, uploaded at create).
struct MeshDev {
  double4* pts64 = nullptr;   // M*6 quadrature points (x,y,z,w*area)
  float4* pts32 = nullptr;
  int4* vid = nullptr;        // M vertex triplets
  double* area = nullptr;     // M
  double* verts = nullptr;    // nv*3
  int32_t* near_rowptr = nullptr;
  int32_t* near_col = nullptr;
  int32_t* near_kind = nullptr;   // 0 identical, 1 edge, 2 vertex
  int32_t* near_vtx = nullptr;    // nnz*6 vertex ids ordered per kind
  double* near_static = nullptr;  // nnz
  double* gl = nullptr;           // Gauss-Legendre nodes (q) then weights (q) on [0,1]
  cf64* s = nullptr;              // F frequencies
  cf64* tw_fwd = nullptr;         // F: zeta^-k
  cf64* tw_inv = nullptr;         // F: zeta^+k
  double* rho_pow = nullptr;      // F: rho^n
  double* rho_ipow = nullptr;     // F: rho^-n / F
  double* ea64 = nullptr;         // Fpad
  double* pb64 = nullptr;
  float* ea32 = nullptr;
  float* pb32 = nullptr;
};

// Offsets (bytes) of the solve workspace.
struct Layout {
  size_t b = 0, ghat = 0, x = 0, r = 0, basis = 0, H = 0, cs = 0, sn = 0, g = 0;
  size_t sysd = 0, sysi = 0, partial = 0, near_val = 0, dense64 = 0, dense32 = 0;
  size_t scratch = 0, total = 0;
  int nsplit = 1;
};

struct H2Operator;  // compressed representation (h2.cpp)

// Optional per-class kernel timing with HIP events recorded on the launch
// stream (enabled by cqm_options.profile).
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> cls;  // class of each recorded pair
  size_t used = 0;       // events used (2 per launch)
  void begin(int c, hipStream_t s);
  void end(hipStream_t s);
  void collect(double* ms, int* calls);  // after the stream is synchronised
  void release();
};

struct Problem {
  Ctx* ctx = nullptr;
  int64_t M = 0, nv = 0;
  int N = 0, F = 0, Fh = 0, Fsys = 0, Fpad = 0, FT = 8;
  double T = 0, dt = 0, rho = 0;
  cqm_options opt{};
  std::vector<double> verts;
  std::vector<int32_t> tris;
  std::vector<double> s_re, s_im;
  // near field (host)
  std::vector<int32_t> rowptr, col, kind, nvtx;
  std::vector<double> static_host;
  bool static_host_valid = false;
  MeshDev dev;
  // incident data
  int inc_kind = 0;  // 0 none, 1 plane wave, 2 samples
  double dir[3] = {1, 0, 0}, sigma = 0.25, t0 = 1.5, amp = 1.0;
  const double* samples = nullptr;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay;
  bool static_ready = false, near_ready = false, dense_ready = false;
  H2Operator* h2 = nullptr;
  cqm_diag last{};
  int64_t far_units = 0;
  KernelTimer timer;
  bool full_band() const { return Fsys == F; }
};

// ------------------------------------------------------------ launchers
// tables / transforms (k_transform.hip)
void launch_rhs(const Problem& p, double* b, hipStream_t s);
void launch_dft_forward(const Problem& p, const double* b, cf64* ghat, hipStream_t s);
void launch_dft_inverse(const Problem& p, const cf64* xhat, double* q, double* imag_sq,
                        double* real_sq, hipStream_t s);
void launch_vec_norms(const cf64* v, int64_t stride, int M, int nsys, double* out, hipStream_t s);
void launch_residual_combine(const cf64* ghat, cf64* r, int M, int nsys, const int* active,
                             hipStream_t s);

// near field (k_near.hip)
void launch_near_static(const Problem& p, hipStream_t s);
void launch_near_values(const Problem& p, cf64* vals, hipStream_t s);
void launch_dense_scatter_near(const Problem& p, const cf64* vals, cf64* d64, cf32* d32,
                               hipStream_t s);

// far field (k_far.hip)
template <typename R>
void launch_far_apply(const Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs,
                      cplx<R>* partial, const int* active, hipStream_t s);
template <typename R>
void launch_far_reduce_near(const Problem& p, int l0, int nsys, const cplx<R>* partial,
                            const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
                            const cf64* near_vals, const int* active, hipStream_t s);
void launch_dense_assemble(const Problem& p, cf64* d64, cf32* d32, hipStream_t s);
int far_partial_slots(int M, int nsys, int precision);  // split-K slots of the far product

// dense products (k_dense.hip)
template <typename R>
void launch_dense_gemv(const cplx<R>* V, int M, int nsys, const cplx<R>* x, int64_t xs,
                       cplx<R>* y, int64_t ys, const int* active, hipStream_t s);

// GMRES (k_gmres.hip)
struct GmresState {
  int M, nsys, m;
  void* basis;      // [nsys][m+1][M] inner precision
  cf64* H;          // [nsys][(m+1)*m]
  double* cs;       // [nsys][m]
  cf64* sn;         // [nsys][m]
  cf64* g;          // [nsys][m+1]
  double* sysd;     // [nsys][8] doubles: 0 beta, 1 tol_abs, 2 bnorm, 3 rnorm
  int* sysi;        // [nsys][4] ints: 0 sys_active, 1 cyc_active, 2 jdone, 3 iters
};
void launch_gmres_init(const cf64* ghat, int M, int nsys, cf64* x, cf64* r, double* sysd,
                       int* sysi, hipStream_t s);
template <typename R>
void launch_cycle_start(const GmresState& st, const cf64* r, double outer_tol, double inner_tol,
                        hipStream_t s);
template <typename R>
void launch_arnoldi(const GmresState& st, int j, hipStream_t s);
template <typename R>
void launch_cycle_finish(const GmresState& st, cf64* x, hipStream_t s);

// ------------------------------------------------------------ host helpers
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w);
void dunavant6(double bary[6][3], double w[6]);
void build_near(Problem& p);
void upload_problem(Problem& p);
void compute_layout(Problem& p);

// RAII helper: times the launches issued in its scope as one class.
struct Timed {
  KernelTimer& t;
  hipStream_t s;
  Timed(Problem& p, int c, hipStream_t st) : t(p.timer), s(st) { t.begin(c, s); }
  ~Timed() { t.end(s); }
};

}  // namespace cqm
