// Internal declarations of the CQM-BEM library (host planner + HIP kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

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
constexpr int kSysiStride = 8; // ints per system in the GMRES status array

// Per-frequency constants of the factor exp(-s r) = 2^(ea r) e^{-2 pi i pb r}:
// ea = -Re(s) log2(e), pb = Im(s) / (2 pi).  Padded with zero-work entries.
template <typename R> struct FreqTab {
  const R* ea;
  const R* pb;
};

// ------------------------------------------------------------ problem state
// GMRES (k_gmres.hip).  One descriptor per frequency system.
// The fields every Arnoldi kernel reads first share the leading 64-byte line
// (one scalar cache line per descriptor fetch).
struct SysDesc {
  int M, m;               // length, restart length
  int prob, l;            // problem index (in a batch) and frequency index
  void* basis;            // (m+1) x M, inner precision
  double* part;           // split Arnoldi: per row slice 4 (m+1) + 2 partial sums
  int* sysi;              // kSysiStride ints of status
  void* symp;             // stored form: tile partials of the product (nt x nt kSymB)
  double* cs;             // m
  cf64* sn;               // m
  cf64* g;                // m+1
  cf64* H;                // (m+1) x m, column-major
  double* sysd;           // 8 doubles of status
  cf64* x;                // M, FP64 solution
  cf64* r;                // M, FP64 residual
  const cf64* ghat;       // M, right-hand side
  const void* V32;        // dense operator slice in FP32 (dense mixed form) or null
  const cf64* V64;        // dense operator slice in FP64 (dense form) or null
  const void* Pinv;       // block-Jacobi inverses (inner precision) or null
  int* hflag;             // pinned host word: the cycle-open flag, written at
                          // every Arnoldi step (or null)
  void* zb;               // where P v_j is formed for the next product: null
                          // for basis slot j + 1 (stored form), else a vector
                          // of its own (matrix-free form: the memory of r,
                          // which the product may not overwrite in place)
};
static_assert(sizeof(SysDesc) == 152, "SysDesc layout");
// Rows per workgroup (one per thread) of the split Arnoldi step.
constexpr int kArnRows = 256;

// Stored operator slices keep the upper triangle of kSymB x kSymB tiles of
// the complex symmetric V(s): tile (I, J), I <= J, at J (J + 1) / 2 + I,
// row-major inside; the last block row/column is padded to kSymB.
constexpr int kSymB = 64;
__host__ __device__ inline int sym_blocks(int M) { return (M + kSymB - 1) / kSymB; }
__host__ __device__ inline int sym_tiles(int M) { return sym_blocks(M) * (sym_blocks(M) + 1) / 2; }
__host__ __device__ inline int64_t sym_slice(int M) { return (int64_t)sym_tiles(M) * kSymB * kSymB; }
// entry (i, j) lives in the stored triangle iff block(i) <= block(j)
__host__ __device__ inline bool sym_stored(int i, int j) { return i / kSymB <= j / kSymB; }
__host__ __device__ inline int64_t sym_index(int i, int j) {
  const int I = i / kSymB, J = j / kSymB;
  return ((int64_t)(J * (J + 1) / 2 + I) * kSymB + i % kSymB) * kSymB + j % kSymB;
}
// partial-sum buffer of one product: nt x (nt kSymB) elements
__host__ __device__ inline int64_t sym_partials(int M) {
  return (int64_t)sym_blocks(M) * sym_blocks(M) * kSymB;
}
// Systems that share one stored operator slice (same mesh, N, T and
// frequency): their products read each row of the slice once.
constexpr int kMaxGroup = 8;
struct GemvGroup {
  int n;
  int sys[kMaxGroup];
};
// A group of systems sharing one stored operator slice, as read by the
// product kernel: everything a workgroup needs hangs off this one record.
struct GroupLite {
  const void* V32;  // FP32 slice (mixed form) or null
  const void* V64;  // FP64 slice
  int M, n;
  float cut32, cut64;      // cut-off radii of the slice's frequency
  const float* gap;        // tile box gaps (cut-off), or null
  long long entries32, entries64;  // entries a product reads under each cut-off
  void* basis[kMaxGroup];  // members' Krylov bases (inner precision)
  cf64* x[kMaxGroup];      // members' FP64 iterates
  void* symp[kMaxGroup];   // members' partial-sum buffers
  int* sysi[kMaxGroup];    // members' status flags
};


// Device tables of the batched GMRES engine (library-owned, grow-only).
struct EngineBufs {
  SysDesc* desc = nullptr;
  size_t desc_cap = 0;
  GroupLite* open_cycle = nullptr;  // groups open at the cycle start
  size_t cycle_cap = 0;
  GroupLite* open_step = nullptr;   // groups with an open cycle
  size_t step_cap = 0;
  GroupLite* staging = nullptr;     // pinned host copies of the two lists
  size_t staging_cap = 0;
  SysDesc* arn_desc = nullptr;      // descriptors of the systems an eager
  size_t arn_cap = 0;               // Arnoldi step runs (open at the last
  SysDesc* arn_staging = nullptr;   // list build), and their pinned staging
  size_t arn_staging_cap = 0;       // (two slots: cycle start, step lists)
  GroupLite* all_groups = nullptr;  // every group (graph-captured steps)
  size_t all_cap = 0;
  GemvGroup* groups = nullptr;
  size_t groups_cap = 0;
  int* status_host = nullptr;       // pinned status flags, written by the device
  int* status_host_dev = nullptr;   // the same buffer's device address
  size_t status_host_cap = 0;
  int* cyc_host = nullptr;          // pinned: [0] step progress, then the
                                    // cycle-open flag of every system
  int* cyc_host_dev = nullptr;
  size_t cyc_cap = 0;
  double* status_norms = nullptr;   // pinned, 3 per system: ||ghat||, last true
  double* status_norms_dev = nullptr;  // residual norm, non-finite flag
};

// Launch shapes picked by timing the candidates on their first use, per
// device context and problem shape (cqm_options.autotune).
struct FarShape {
  int ft = 0;        // frequencies per workgroup
  int waves = 4096;  // waves the source split aims for
};
struct Tuner {
  std::mutex mu;
  std::map<uint64_t, FarShape> far;  // (M, systems, precision)
  std::map<uint64_t, int> assemble;  // (M, systems) -> frequency tile
};

// One problem of a work-queue assembly launch (k_far.hip): its tables and
// outputs, cut-off exponents, and its items [item0, item0 + tiles nft).
struct AsmJob {
  const double4* pts;
  const int4* vid;
  const double* ea;
  const double* pb;
  cf64* d64;
  cf32* d32;
  const int32_t* nrp;
  const int32_t* ncol;
  const cf64* nval;
  const double* sbox;
  int64_t nnz;
  long long item0;
  int M, nsys, nft, pad;
  double Lin, Lout;
};

struct Ctx {
  int device = 0;
  int cus = 256;  // compute units of the device
  EngineBufs eb;
  Tuner tune;
  // work-queue assembly: job table and item counter (grow-only)
  AsmJob* asm_jobs = nullptr;
  AsmJob* asm_stage = nullptr;  // pinned host copy the table is uploaded from
  size_t asm_cap = 0;
  unsigned long long* asm_counter = nullptr;
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
  int32_t* near_row = nullptr;    // row of each near pair
  int32_t* near_kind = nullptr;   // 0 identical, 1 edge, 2 vertex
  int32_t* near_vtx = nullptr;    // nnz*6 vertex ids ordered per kind
  double* near_static = nullptr;  // nnz
  double* gl = nullptr;           // Gauss-Legendre nodes (q) then weights (q) on [0,1]
  cf64* s = nullptr;              // F frequencies
  cf64* tw_fwd = nullptr;         // F: zeta^-k
  cf64* tw_inv = nullptr;         // F: zeta^+k
  double* rho_pow = nullptr;      // F: rho^n
  double* rho_ipow = nullptr;     // F: rho^-n / F
  double* ftab = nullptr;         // FP64 exp/sincos tables (2^(j/256), (sin, cos)(2 pi j/256))
  double* ea64 = nullptr;         // Fpad
  double* pb64 = nullptr;
  double* ea64u = nullptr;        // ea64 in steps of ln2/256, pb64 in steps of 2 pi/512
  double* pb64u = nullptr;
  float* ea32 = nullptr;
  float* pb32 = nullptr;
  // cut-off tables: per stored 64 x 64 tile (I, J), the gap between the
  // bounding boxes of the two blocks' triangles (sym_tiles(M) floats, tile
  // order of the packed triangle); per 16-triangle group of the assembly
  // tiling, its box lo[3], hi[3]
  float* tile_gap = nullptr;
  double* sub_box = nullptr;
  // double-layer operator (direct formulation): unit normals of the
  // triangles (vertex order), the static near part of K (nnz)
  double4* nrm64 = nullptr;
  double* nearK_static = nullptr;
  double* nearD_static = nullptr;  // nnz*9: hypersingular static weights [a][b] (direct formulation)
  int32_t* v2t_ptr = nullptr;      // nv+1: vertex -> (triangle, local vertex) slots
  int32_t* v2t = nullptr;          // 3M slots 3*i + a, ascending per vertex
  int32_t* near_tpos = nullptr;   // nnz: position of pair (j, i) for pair (i, j)
};
// Frequency-dependent cut-off radii of a system: tiles whose box gap is at
// least cut32 (inner precision) or cut64 (FP64 operator) are left out.
inline float cutoff_radius(double L, double re_s) {
  return (L > 0.0 && re_s > 0.0) ? (float)(L / re_s) : 3.0e38f;
}

// Offsets (bytes) of the solve workspace.
struct Layout {
  size_t partial = 0, near_val = 0, dense64 = 0, dense32 = 0, pinv = 0, diag64 = 0, total = 0;
  // compressed modes with refine_plain: split-K partial sums of the FP64
  // matrix-free product that forms the refinement residuals
  size_t mfpart = 0;
  // direct formulation: near values of K (nnz x Fsys), the coefficient
  // vectors it is applied to (Fsys x M) and its split-K partial sums
  size_t nearK = 0, kin = 0, kpart = 0, dsrc = 0, dz = 0, dpart = 0;
  // time marching (cqm_options.marching): weights, What_0 block inverses and
  // their complex staging, product partials, CG vectors and partial sums
  size_t mw = 0, mpinv = 0, mdiag = 0, mpart = 0, mvec = 0;
  // compressed time marching: past densities as complex rows (newest last),
  // the history product's outputs, the CG product's input and output
  size_t mz = 0, my = 0, mpc = 0;
  int mchunks = 1;  // weight chunks of the history product (its partial slots)
};

struct H2Operator;  // compressed representation (h2.cpp)
struct Problem;

// Incident Dirichlet data of one right-hand side.
struct Incident {
  int kind = 0;  // 0 none, 1 plane wave, 2 samples at the quadrature points
  double dir[3] = {1, 0, 0}, sigma = 0.25, t0 = 1.5, amp = 1.0;
  const double* samples = nullptr;  // device, (N+1) x M x 6
};

// Per-right-hand-side solve state: data samples, transforms, Krylov basis,
// Hessenberg data and status of every frequency system.  Offsets are bytes
// from `base`.  A problem owns one in its workspace; the serving loop adds
// more that share the problem's operator.
struct SolveState {
  Problem* p = nullptr;
  char* base = nullptr;
  size_t b = 0, ghat = 0, x = 0, r = 0, basis = 0, H = 0, cs = 0, sn = 0, g = 0, sysd = 0,
         sysi = 0, part = 0, sym = 0, scratch = 0, total = 0;
  Incident inc;
  double* q_out = nullptr;
  cqm_diag diag{};
  int first = 0;  // index of its first system in the engine's descriptor list
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
};

// Optional per-class kernel timing with HIP events recorded on the launch
// stream, and per-class algorithmic work counted by the kernels themselves
// (one device atomic per workgroup), both enabled by cqm_options.profile.
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  std::vector<int> cls;  // class of each recorded pair
  size_t used = 0;       // events used (2 per launch)
  unsigned long long* work_d = nullptr;  // CQM_K_CLASSES device counters
  void begin(int c, hipStream_t s);
  void end(hipStream_t s);
  void reset(hipStream_t s);             // clear events and counters
  unsigned long long* ctr(int c) const { return on && work_d ? work_d + c : nullptr; }
  // after the stream is synchronised
  void collect(double* ms, int* calls, double* work);
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
  // incident data and the problem's own solve state
  Incident inc;
  SolveState own;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay;
  bool static_ready = false, near_ready = false, dense_ready = false;
  bool nearK_static_ready = false, nearK_ready = false, nearD_static_ready = false;
  H2Operator* h2 = nullptr;
  cqm_diag last{};
  int64_t far_units = 0;
  KernelTimer timer;
  // engine of the problem's own solves, kept across them (with its buffers
  // and captured step graphs)
  class Engine* engine = nullptr;
  hipEvent_t setup_ev[2] = {nullptr, nullptr};  // brackets the operator setup of a solve
  EngineBufs engine_bufs;
  int* march_host = nullptr;  // pinned: [0] converged flag, [1] step iterations
  // stored-form entries a product reads per frequency under the inner and
  // the FP64 cut-off (upper triangle; filled on first use)
  std::vector<int64_t> cut_entries32, cut_entries64;
  std::vector<float> tile_gap_host;  // host copy of dev.tile_gap
  bool full_band() const { return Fsys == F; }
};

// ------------------------------------------------------------ launchers
// tables / transforms (k_transform.hip)
void launch_rhs(const Problem& p, const Incident& inc, double* b, hipStream_t s);
// (also clears zero2[0..1], the inverse transform's accumulators, if given)
void launch_dft_forward(const Problem& p, const double* b, cf64* ghat, double* zero2,
                        hipStream_t s);
void launch_dft_inverse(const Problem& p, const cf64* xhat, double* q, double* imag_sq,
                        double* real_sq, hipStream_t s);
void launch_vec_norms(const cf64* v, int64_t stride, int M, int nsys, double* out, hipStream_t s);

// near field (k_near.hip)
void launch_near_static(const Problem& p, hipStream_t s);
void launch_near_values(const Problem& p, cf64* vals, hipStream_t s);

// far field (k_far.hip)
template <typename R>
void launch_far_apply(const Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs,
                      cplx<R>* partial, const int* active, unsigned long long* ctr, hipStream_t s);
template <typename R>
void launch_far_reduce_near(const Problem& p, int l0, int nsys, const cplx<R>* partial,
                            const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
                            const cf64* near_vals, const int* active, hipStream_t s);
// all frequency slices of the packed operator: far entries evaluated, near
// ones (pairs sharing a vertex) copied from the near-field values nv
void launch_dense_assemble(const Problem& p, cf64* d64, cf32* d32, const cf64* nv,
                           unsigned long long* ctr, hipStream_t s);
// Records msg as the calling thread's cqm_last_error() and returns code.
int fail_with(int code, const std::string& msg);
// Double-layer operator K(s) (k_dlayer.hip): static near part, near values
// per frequency, y = alpha z + K x (z may be y; FP64, matrix-free far field),
// and c = g / area.
void launch_nearK_static(const Problem& p, hipStream_t s);
void launch_nearK_values(const Problem& p, cf64* vals, hipStream_t s);
void launch_apply_K(const Problem& p, int l0, int nsys, const cf64* x, int64_t xs, const cf64* z,
                    double alpha, cf64* y, int64_t ys, const cf64* nvals, cf64* partial,
                    bool adjoint, hipStream_t s);
void launch_div_area(const Problem& p, int nsys, const cf64* g, int64_t gs, cf64* c, hipStream_t s);
size_t dl_partial_bytes(int M, int Fs);
// hypersingular operator (k_hsing.hip): the barycentric coordinates of the
// 6-point rule's points, passed by value to the kernels
struct HsRule {
  double bary[6][3];
};
size_t hs_partial_bytes(int M, int Fs);
void launch_nearD_static(const Problem& p, hipStream_t s);
void launch_apply_D(const Problem& p, int l0, int nsys, const cf64* x, int64_t xs, cf64* y,
                    int64_t ys, cf64* src, cf64* partial, cf64* z, hipStream_t s);
int far_partial_slots(int M, int nsys, int precision);  // split-K slots of the far product (any shape)
// Allocation-free far product (matrix-free form): partial sums in the fixed
// device array of kFarScratchBytes (k_far.hip), whose address is looked up
// once per device by far_scratch_init (with that device current).
constexpr size_t kFarScratchBytes = size_t(64) << 20;
void far_scratch_init(int device);
template <typename R>
void launch_far_apply_fixed(const Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs,
                            cplx<R>* y, int64_t ys, const cf64* near_vals, hipStream_t s);
FarShape far_shape_of(const Problem& p, int nsys, int precision);  // shape in use (tuned or default)

// dense products (k_dense.hip)
template <typename R>
void launch_dense_gemv(const cplx<R>* V, int M, int nsys, const cplx<R>* x, int64_t xs,
                       cplx<R>* y, int64_t ys, const int* active, cplx<R>* part, hipStream_t s);

void launch_gmres_init(const SysDesc* sd, int n, hipStream_t s);
void launch_residual_combine(const SysDesc* sd, int n, hipStream_t s);

// flags (kSysiStride ints) and ||ghat||, last residual norm, non-finite flag
// (3 doubles) of n systems, into host-visible memory
void launch_gather_diag(const SysDesc* sd, int n, int* flags, double* norms, hipStream_t s);
// relax > 0: inexact refinement (the inner target follows the reduction of
// the last cycle, for inner operators that approximate the outer one)
template <typename R>
void launch_cycle_start(const SysDesc* sd, int n, double outer_tol, double inner_tol, double relax,
                        hipStream_t s);
// split: three launches over row slices; fused (split only): the first one
// also sums the stored-operator partials of w = A v_j (no separate reduction)
template <typename R>
void launch_arnoldi(const SysDesc* sd, int n, int maxM, int j, bool split, bool fused,
                    bool pre, unsigned long long* ctr, int* prog, hipStream_t s);
template <typename R> void launch_cycle_finish(const SysDesc* sd, int n, int maxM, hipStream_t s);
// dense products over descriptors (k_dense.hip): which = 0 inner product
// basis[j] -> basis[j+1] of systems with an open cycle; which = 1 FP64
// residual product x -> r of open systems.  rowmap: (system, first row).
template <typename R>
void launch_dense_gemv_groups(const GroupLite* gl, int ngroups, int M, bool grouped, int which,
                              int j, unsigned long long* ctr, hipStream_t s);
template <typename R>
void launch_dense_reduce_desc(const SysDesc* sd, int nsys, int maxM, int which, int j,
                              hipStream_t s);
// FP64 refinement residuals r = ghat - V x of the stored form in
// double-double arithmetic (partials as (hi, lo): 2 sym_partials cf64 per
// system), for systems with an open outer iteration
void launch_resid_dd_groups(const GroupLite* gl, int ngroups, int M, bool grouped,
                            unsigned long long* ctr, hipStream_t s);
void launch_resid_dd_reduce(const SysDesc* sd, int nsys, int maxM, hipStream_t s);
// Block-Jacobi preconditioner (k_dense.hip): inverses of the kSymB x kSymB
// diagonal blocks of every slice (elimination and storage in R), from the
// packed slice's diagonal tiles or from a compact array of the blocks;
// application z = P v_j into basis slot j+1 (or zb) for systems with an open
// cycle.  (The FP32 finish kernel forms the next step's z itself, the cycle
// finish x += P V y.)
template <typename R>
void launch_block_inverse(const cf64* d64, int M, int nsys, bool compact, cplx<R>* pinv,
                          hipStream_t s);
// the diagonal kSymB-blocks of every V(s_l), FP64, compact [l][block][row][col]
// (block-Jacobi preconditioner of the matrix-free form; k_far.hip)
void launch_diag_blocks(const Problem& p, cf64* d, const cf64* nv, hipStream_t s);
// the stored operators of several problems (same context) in one persistent
// work-queue launch; each problem's d64 / d32 / near values as in
// launch_dense_assemble
void launch_dense_assemble_batch(const std::vector<Problem*>& ps, const std::vector<cf64*>& d64,
                                 const std::vector<cf32*>& d32, const std::vector<const cf64*>& nv,
                                 unsigned long long* ctr, hipStream_t s);
template <typename R>
void launch_block_apply(const SysDesc* sd, int n, int maxM, int j, hipStream_t s);
inline int64_t block_inverse_elems(int M) { return (int64_t)sym_blocks(M) * kSymB * kSymB; }

// ------------------------------------------------------------ host helpers
void gauss_legendre01(int q, std::vector<double>& x, std::vector<double>& w);
void dunavant6(double bary[6][3], double w[6]);
void build_near(Problem& p);
void upload_problem(Problem& p);
void compute_layout(Problem& p);
size_t state_layout(const Problem& p, SolveState& st);  // offsets of a state; returns bytes
bool mode_is_mixed(int mode);
bool mode_is_h2(int mode);

// solve driver (engine.cpp)
template <typename R>
void apply_op(Problem& p, int l0, int nsys, const cplx<R>* x, int64_t xs, cplx<R>* y, int64_t ys,
              const int* active, hipStream_t s);
void prepare_operator(Problem& p, hipStream_t s);
void prepare_double_layer(Problem& p, hipStream_t s);  // near values of K (direct formulation)
// timed: measure the setup with the problem's events instead of a stream
// synchronisation (one caller per problem at a time)
void pre_solve(SolveState& st, hipStream_t s, bool prepare, bool timed = false);
void post_solve(SolveState& st, hipStream_t s);
int diag_status(const cqm_diag& dg);  // CQM_OK / CQM_ENOCONV / CQM_ENAN
void solve_states(std::vector<SolveState*>& S, hipStream_t s);  // full solves, grouped by precision

// One restart cycle at a time over a changing set of states (same inner
// precision): used by the batch solve and by the serving loop.
class Engine {
 public:
  explicit Engine(Ctx& c) : eb(c.eb) {}
  Engine(Ctx&, EngineBufs& b) : eb(b) {}  // own descriptor/status buffers
  ~Engine();
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;
  void set(const std::vector<SolveState*>& S, hipStream_t s);  // rebuild descriptors
  void init(int k, hipStream_t s);                              // x = 0, r = ghat of state k
  int cycle(hipStream_t s);                                     // returns systems still open
  void status(hipStream_t s);                                   // refresh host flags
  bool state_done(int k) const;                                 // every system of state k closed
  // fill diag of state k (refresh: recompute the residual norms first)
  void finish_diag(int k, hipStream_t s, bool refresh = true);
  int cycles_run = 0;
  bool mixed = true;
 private:
  template <typename R> int cycle_t(hipStream_t s);
  EngineBufs& eb;
  std::vector<SolveState*> S_;
  std::vector<SysDesc> hd_;
  std::vector<GroupLite> lite_;   // one record per stored-operator group
  struct GClass {                 // open groups of one mesh size in a device list
    int M, off, count;
    bool grouped;
  };
  std::vector<GClass> cyc_cls_, step_cls_;
  // groups with a member whose flag `which` is set (host flags), by mesh
  // size, uploaded to dst from the pinned staging area at `stage`
  // descriptors of the systems with an open cycle into eb.arn_desc (staging
  // slot 0 at a cycle start, 1 at later list builds); the eager Arnoldi
  // steps run over them only, so closed systems issue no loads
  void upload_arnoldi(int slot, hipStream_t s);
  int arn_n_ = 0;
  void upload_open(int which, GroupLite* dst, size_t stage, std::vector<GClass>& cls,
                   hipStream_t s);
  // reduce = false leaves the partial sums for the Arnoldi step to add up
  template <typename R>
  void dense_product(const GroupLite* list, const std::vector<GClass>& cls, int which, int j,
                     bool reduce, unsigned long long* ctr, hipStream_t s);
  std::vector<GemvGroup> groups_;
  bool split_ = false;    // Arnoldi step split over row slices
  bool prev_split_ = false;  // layout the captured steps were recorded with
  // block-Jacobi right preconditioning of the stored-operator systems: each
  // step forms P v_j before the product, each cycle closes with x += P V y
  // pre_: the stored-form products read slot j + 1; anypre_: some system
  // (either form) is preconditioned
  bool pre_ = false, anypre_ = false, prev_pre_ = false;
  // FP32 split steps form P v_{j+1} inside the Arnoldi finish kernel; only
  // the first step of a cycle launches the block product itself
  template <typename R> bool fuse_pre() const { return anypre_ && split_ && sizeof(R) == 4; }
  std::vector<int> flags_;
  int maxM_ = 0, m_ = 30;
  // inside a cycle the host queues step j + 1 once the last kernel of step
  // j - kAhead has started (progress word) and reads the cycle-open flags
  // after queueing each step.  0 measured best at C2 (3.21 ms per solve,
  // against 3.24 / 3.29 / 3.35 / 3.55 ms for 1 / 2 / 3 / 5): every step
  // queued beyond a cycle's last useful one costs a full launch sequence,
  // while issuing a step takes the host less time than the kernel it waits on
  static constexpr int kAhead = 0;
  void wait_progress(int target, hipStream_t s);
  // HIP graphs of the Arnoldi steps (dense-form batches without profiling):
  // step j = products of every group + the Arnoldi step, over the full group
  // list (closed systems are skipped inside the kernels).  Captured on first
  // use and kept while set() rebuilds the same descriptors.
  bool graphs_ = false;
  hipStream_t cap_stream_ = nullptr;
  std::vector<GClass> all_cls_;
  std::vector<hipGraphExec_t> gexec_;
  std::vector<SysDesc> prev_hd_;
  void drop_graphs();
  template <typename R> void step_eager(int j, const GroupLite* list, const std::vector<GClass>& cls,
                                        hipStream_t s);
  template <typename R> void step_graph(int j, hipStream_t s);
};

void release_engine_bufs(EngineBufs& b);

// ------------------------------------------------------------ time marching
// Vectors and partial sums of the conjugate gradients on What_0 (k_march.hip).
struct CgVec {
  double *x, *r, *z, *p, *w;
  double *rz, *pw, *rr, *bb;  // per-workgroup partials (rz by iteration parity)
  int* done;                  // device flag: converged
  int* hdone;                 // pinned host flag (the host polls it)
  int* iters;                 // pinned host counter: iterations of the step
  const cf64* pinv;           // block inverses of What_0 (real parts used)
  int M, nwg;
};
void launch_march_weights(const cf64* V, int M, int H, int F, const cf64* tw, const double* scale,
                          double* W, hipStream_t s);
int march_chunks(int M, int cnt);
void launch_march_product(const double* W, int M, int j0, int cnt, const double* X, int xb,
                          double* P, int S, const int* done, hipStream_t s);
void launch_march_reduce(const double* P, int S, int M, double sign, const double* add, double* y,
                         hipStream_t s);
void launch_march_diag(const double* W0, int M, cf64* out, hipStream_t s);
void launch_cg_init(const CgVec& v, hipStream_t s);
void launch_cg_iteration(const CgVec& v, const double* W0, double* P, int par, double tol2,
                         hipStream_t s);
void solve_marching(Problem& p, double* q_out, cqm_diag* diag, hipStream_t s);  // march.cpp
// compressed time marching (h2.cpp): the weights What_n from the fibres, and
// y_k = What_k x_k for k = k0 .. k0+nsys-1 (complex in and out)
void h2_marching_weights(Problem& p, hipStream_t s);
void h2_apply_weights(Problem& p, int k0, int nsys, const cf64* x, int64_t xs, cf64* y, int64_t ys,
                      hipStream_t s);
// fast right-hand side (eq. fastrhs): record step m's input x (complex,
// triangle order) as history row hx (cluster order) with its cluster
// coefficients; y = sum_{k=1}^{n} What_k x_{n-k} from rows 0 .. n-1
void h2_history_push(Problem& p, int m, const cf64* x, cf64* hx, hipStream_t s);
void h2_history_sum(Problem& p, int n, const cf64* hx, cf64* y, hipStream_t s);
// compressed marching helpers (k_march.hip): r = b - Re sum_{k<n} Y[k];
// Z = x as complex; w = Re Y with the partial p.w (CG product); the mean
// over the frequencies of the plain diagonal blocks (real part)
void launch_hist_reduce(const cf64* Y, int n, int M, const double* b, double* r, hipStream_t s);
void launch_to_complex(const double* x, int M, cf64* z, const int* done, hipStream_t s);
void launch_cg_reduce_complex(const CgVec& v, const cf64* y, hipStream_t s);
void launch_freq_mean_blocks(const cf64* blocks, int F, int64_t nel, cf64* out, hipStream_t s);
void launch_cg_check(const CgVec& v, double tol2, hipStream_t s);
void launch_cg_finish(const CgVec& v, int par, hipStream_t s);

// RAII helper: a named host range around a stage (rocprofv3 --marker-trace
// records it; without a profiler the calls return at once).
struct Stage {
  explicit Stage(const char* name) { roctxRangePushA(name); }
  ~Stage() { roctxRangePop(); }
  Stage(const Stage&) = delete;
  Stage& operator=(const Stage&) = delete;
};

// RAII helper: times the launches issued in its scope as one class.
struct Timed {
  KernelTimer& t;
  hipStream_t s;
  Timed(Problem& p, int c, hipStream_t st) : t(p.timer), s(st) { t.begin(c, s); }
  ~Timed() { t.end(s); }
};

}  // namespace cqm

// Opaque handle types of the C ABI.
struct cqm_ctx_s : cqm::Ctx {};
struct cqm_problem_s : cqm::Problem {};
