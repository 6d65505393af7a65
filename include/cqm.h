/*
 * cqm.h -- C ABI of the MI355X library for time-domain single-layer BEM by
 * convolution quadrature (all-at-once form), with optional H2 x MACA
 * compression of the space x space x frequency operator tensor.
 *
 * Method (Seibel, "Boundary Element Methods for the Wave Equation based on
 * Hierarchical Matrices and Adaptive Cross Approximation"):
 *   - frequencies s_l = delta(rho zeta^-l)/dt of the BDF2 convolution
 *     quadrature, zeta = exp(2 pi i/(N+1))          (Section 3.1, eq. cqm_freq)
 *   - Galerkin single-layer matrices V(s_l) on piecewise-constant elements,
 *     kernel exp(-s|x-y|)/(4 pi |x-y|)                (Section 3.2, eq. fundsol)
 *   - N+1 independent systems V(s_l) xhat_l = ghat_l, ghat/xhat linked to the
 *     time steps by scaled DFTs                       (remark ending Section 6.2)
 *   - optional compression: H2 in space (Section 4, Algorithm 1) and
 *     multivariate ACA across frequencies (Section 5, Algorithms 2 and 3).
 *   - the other operators of the Calderon system (Section 2.2, eq. wavebio)
 *     per frequency: the double layer K and its adjoint K' on
 *     piecewise-constant elements, the hypersingular D on piecewise-linear
 *     ones, and the direct Dirichlet formulation (eq. wavegalform).
 *
 * Conventions
 *   - Every function returns int: 0 on success or a negative CQM_E* code.
 *     cqm_last_error() returns a thread-local message for the last failure.
 *   - The caller owns every input and output buffer and the solve workspace.
 *     The library owns handles (freed by the matching _destroy) and the small
 *     per-mesh tables it uploads at cqm_problem_create.
 *   - Pointers are DEVICE pointers unless the parameter says "host".
 *   - Calls taking a hipStream_t enqueue on that stream.  cqm_solve and
 *     cqm_solve_batch synchronise that stream internally (convergence is
 *     steered by flags the device writes to host memory) and return when the
 *     output is written; cqm_apply_V returns once its launches are queued.
 *   - Each declaration names the passage of the paper that defines what it
 *     computes, or says "Paper: no passage" for plumbing.
 *   - Complex device arrays are interleaved (re, im) pairs of double
 *     (precision 64) or float (precision 32).
 *   - Time-step arrays are row-major (N+1) x M: row n is t_n = n*dt, column i
 *     is triangle i in the caller's triangle order.
 */
#ifndef CQM_H
#define CQM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define CQM_OK 0
#define CQM_EINVAL (-1)  /* bad mesh, sizes, options or arguments            */
#define CQM_ENOMEM (-2)  /* workspace missing/too small or HBM budget exceeded */
#define CQM_ENOCONV (-3) /* some frequency missed its tolerance; output and
                            diagnostics are still written                     */
#define CQM_ENAN (-4)    /* NaN/Inf in the data or the iteration            */
#define CQM_EDEVICE (-5) /* HIP runtime failure                              */

/* ------------------------------------------------------------ options */
/* Precision / representation of the operator. */
#define CQM_FP64_PLAIN 0   /* FP64 kernel evaluation, FP64 GMRES            */
#define CQM_MIXED_PLAIN 1  /* FP32 inner GMRES, FP64 outer residuals.  The
                              near-field entries are computed in FP64; the
                              matrix-free form also applies them in FP64,
                              while the stored form keeps one FP32 copy of
                              the whole operator (near entries included) for
                              the inner products and the FP64 one for the
                              residuals                                      */
#define CQM_MIXED_H2ACA 2  /* H2 x MACA operator, FP32-stored factors in the
                              inner solve, FP64 residuals                    */
#define CQM_FP64_H2ACA 3   /* H2 x MACA operator, all FP64                    */

/* Storage of the plain operator. */
#define CQM_FORM_MATRIX_FREE 0 /* kernel evaluated on the fly in every product */
#define CQM_FORM_DENSE 1       /* all V(s_l) assembled once in HBM           */

/* Frequency band handled by MACA (V(conj s) = conj V(s): the half band
   and conjugation give the rest). */
#define CQM_BAND_FULL 0 /* all N+1 frequencies compressed and solved */
#define CQM_BAND_HALF 1 /* l = 0..N/2 solved, the rest by conjugation */

typedef struct cqm_options {
  int32_t mode;          /* CQM_FP64_PLAIN ...                       (1)    */
  int32_t form;          /* CQM_FORM_* for plain modes               (DENSE) */
  double rho;            /* contour radius; 0 selects rho^N = 1e-8          */
  int32_t gmres_restart; /* Krylov dimension per cycle               (30)   */
  int32_t max_cycles;    /* restart cycles; each restarts from the FP64
                            true residual                            (60)   */
  double inner_tol;      /* relative residual reduction per cycle    (1e-8),
                            floored at 2e-7 when the cycle runs in FP32    */
  double outer_tol;      /* FP64 relative residual per frequency     (1e-15);
                            a restart that no longer halves a residual
                            already below 1e-13 also ends the system     */
  int32_t n_min;         /* cluster leaf size                        (32)   */
  double eta;            /* box admissibility parameter              (1.0)  */
  int32_t cheb_m;        /* Chebyshev points per axis, rank m^3, 2..8 (4)   */
  double eps_aca;        /* MACA stopping tolerance                  (1e-6) */
  int32_t aca_band;      /* CQM_BAND_*                               (FULL) */
  int32_t q_duffy;       /* Gauss points per Duffy dimension (<= 16) (5)    */
  int32_t reuse_operator;/* nonzero: keep the assembled operator between
                            solves of the same problem                (0)   */
  int32_t profile;       /* nonzero: time kernel classes with HIP events
                            on the solve stream (cqm_diag.kernel_ms)  (0)   */
  int32_t arnoldi_layout;/* CQM_ARNOLDI_*: workgroups per system in the
                            Arnoldi step                             (AUTO) */
  int32_t autotune;      /* nonzero: time the launch-shape candidates of
                            the far product and the dense assembly on
                            their first use per context and problem
                            shape, keep the fastest (one host wait)  (1)   */
  int32_t graphs;        /* nonzero: Arnoldi steps of stored-form solves
                            without profiling replay captured HIP graphs
                            (kept across solves of the same problem; the
                            full group list is used, so closed groups are
                            launched and leave at once)               (0)   */
  int32_t precond;       /* CQM_PRECOND_*: right preconditioner of the
                            inner GMRES for the plain forms: the inverses
                            of the 64 x 64 diagonal blocks of every
                            V(s_l), formed once per operator (stored form:
                            from its diagonal tiles; matrix-free form:
                            those blocks assembled on their own, 16 B per
                            entry plus the inverses).  It does not change
                            the solution (the refinement residual is the
                            unpreconditioned one), only the number of
                            inner steps; the compressed modes use the
                            plain operator's diagonal blocks the same way
                            (the near-field values they need as well).
                                                                (BLOCK_JACOBI) */
  int32_t marching;      /* nonzero: the workspace also holds the real
                            integration weights What_n, n = 0..N, of the
                            stored form (N+1 slices of the packed
                            triangle, 8 B per entry), or for a compressed
                            mode the transformed fibres, What_0 densely
                            (8 M^2 B) and the history of past densities,
                            for cqm_solve_marching                    (0)   */
  double cutoff_inner;   /* cut-off of the stored form's inner-iteration
                            (FP32) operator: a 64 x 64 tile (16 x 16 in the
                            assembly) is left out of frequency l when
                            Re(s_l) r_min >= cutoff_inner, r_min the gap of
                            the tiles' bounding boxes, so every entry left
                            out is below e^-cutoff_inner of the kernel
                            scale (introduction: cut-off strategies);
                            0 = off                                   (18) */
  double cutoff_outer;   /* the same for the FP64 operator (assembly and
                            refinement residuals); 45 leaves out entries
                            below 3e-20 of the kernel scale, far under FP64
                            rounding; 0 = off                         (45) */
  int32_t refine_plain;  /* compressed modes: nonzero forms every FP64
                            refinement residual with the plain operator
                            (the FP64 matrix-free product of Section 3.2's
                            Galerkin entries plus the near-field values),
                            so the answer is the plain method's to
                            outer_tol and the compressed operator only
                            carries the inner iterations; 0 forms it with
                            the compressed operator, whose approximation
                            error (Section 6.1: m, eta, eps_aca) then
                            stays in the answer.  With refine_plain the
                            inner target of a cycle after the first is
                            0.1 x the previous cycle's residual reduction
                            (at most 1e-3, never below inner_tol)      (1) */
  int32_t formulation;   /* CQM_FORMULATION_*: the boundary integral
                            equation solved                     (INDIRECT) */
} cqm_options;

/* Formulations (cqm_options.formulation).  INDIRECT: V phi = g_D, phi a
   single-layer density (q_out is phi).  DIRECT: the Galerkin equation of
   Section 2.2 (eq. wavegalform) for a Dirichlet boundary, V q =
   (-1/2 I + K) g_D with K the double-layer operator (eq. wavebio), q_out the
   Neumann datum; g_D is represented by its L2 projection onto piecewise
   constants (the paper uses piecewise linears), K is applied once per solve
   (FP64, matrix-free).  The marching solve takes INDIRECT only. */
#define CQM_FORMULATION_INDIRECT 0
#define CQM_FORMULATION_DIRECT 1

/* Inner preconditioners (cqm_options.precond). */
#define CQM_PRECOND_NONE 0
#define CQM_PRECOND_BLOCK_JACOBI 1

/* Arnoldi step layouts (cqm_options.arnoldi_layout).  AUTO splits when a
   batch has fewer systems than the GPU has compute units (256). */
#define CQM_ARNOLDI_AUTO 0   /* choose by the number of systems            */
#define CQM_ARNOLDI_GROUP 1  /* one workgroup per system, one launch      */
#define CQM_ARNOLDI_SPLIT 2  /* ceil(M/256) workgroups per system, three
                                launches (dots, update, finish)           */

/* Kernel classes timed when cqm_options.profile is set. */
#define CQM_K_FAR32 0    /* matrix-free far-field product, FP32          */
#define CQM_K_FAR64 1    /* matrix-free far-field product, FP64          */
#define CQM_K_ASSEMBLE 2 /* dense FP64 assembly of all V(s_l), or MACA  */
#define CQM_K_GEMV32 3   /* stored or compressed operator products, inner
                            precision                                    */
#define CQM_K_GEMV64 4   /* stored or compressed operator products, FP64 */
#define CQM_K_NEAR 5     /* near-field static and per-frequency parts    */
#define CQM_K_ARNOLDI 6  /* Arnoldi step: orthogonalisation, Givens      */
#define CQM_K_OTHER 7    /* right-hand side, DFTs, GMRES restart/update
                            bookkeeping, compression kernels             */
#define CQM_K_CLASSES 8

/* Diagnostics of one solve (host struct). */
typedef struct cqm_diag {
  int32_t n_systems;        /* frequencies solved                          */
  int32_t cycles;           /* restart cycles run                          */
  int32_t total_iters;      /* Arnoldi steps summed over frequencies       */
  int32_t max_iters;        /* Arnoldi steps of the slowest frequency      */
  double max_rel_residual;  /* max_l ||ghat_l - V_l xhat_l|| / ||ghat_l||  */
  double imag_ratio;        /* ||Im q|| / ||Re q|| before taking Re       */
  double t_setup_ms;        /* near field + operator assembly / compression */
  double t_solve_ms;        /* RHS, transforms and GMRES                   */
  int64_t operator_bytes;   /* device bytes of the operator representation */
  int32_t converged;        /* 1 if every frequency met outer_tol          */
  int32_t max_rank;         /* MACA: largest block rank                    */
  double mean_rank;         /* MACA: mean block rank                       */
  int32_t n_far_blocks;     /* H2: admissible blocks                       */
  int32_t n_near_blocks;    /* H2: inadmissible leaf blocks                */
  int64_t far_units;        /* point-pair-frequency kernel values per plain
                               far-field product (matrix-free form)        */
  double kernel_ms[8];      /* GPU time per CQM_K_* class (profile only)   */
  int32_t kernel_calls[8];  /* launches per CQM_K_* class (profile only)   */
  int32_t far_tile;         /* frequencies per workgroup of the matrix-free
                               far product (inner precision) in use       */
  int32_t far_waves;        /* waves its source split aims for           */
  double kernel_work[8];    /* algorithmic work per CQM_K_* class, counted
                               by the kernels (profile only): FAR32, FAR64
                               and ASSEMBLE in point-pair-frequency kernel
                               values evaluated; GEMV32, GEMV64 and ARNOLDI
                               in bytes the algorithm must move (operator
                               rows once, Krylov vectors per pass); others 0 */
  int64_t h2_plain_bytes;   /* H2 x MACA: bytes of the same blocks without
                               the frequency compression (every block's
                               spatial factor per frequency, plus the
                               bases): plain H2 storage, Section 7.1     */
  int32_t reserved[4];
} cqm_diag;

typedef struct cqm_ctx_s* cqm_ctx_t;
typedef struct cqm_problem_s* cqm_problem_t;
typedef struct cqm_server_s* cqm_server_t;

/* Thread-local message describing the last error (never NULL).
 * Paper: no passage (error reporting of the library). */
const char* cqm_last_error(void);

/* Fill *opt (host) with the defaults listed above.  The method parameters
 * follow Section 3.1 (rho, eq. cqm_freq), Section 4.1 (n_min, eta,
 * eq. qadm), Section 4.2 (cheb_m, Algorithm 1) and Section 5.1 (eps_aca,
 * Algorithm 2); the solver parameters are this library's (the paper solves
 * by LU, Section 3.2, and suggests iterative solvers, Section 6.2).
 * CQM_EINVAL if opt is NULL. */
int cqm_default_options(cqm_options* opt);

/* ------------------------------------------------------------ context */
/* Bind a context to HIP device `device` (library-owned handle, freed by
 * cqm_ctx_destroy after every problem and server on it).  CQM_EINVAL for a
 * bad device index or NULL out.  Paper: no passage (device binding). */
int cqm_ctx_create(int device, cqm_ctx_t* out);
int cqm_ctx_destroy(cqm_ctx_t ctx);

/* ------------------------------------------------------------ problems */
/* Create a problem on a closed surface mesh: the flat triangles and the
 * piecewise-constant space S_h^0 of Section 3.2, N steps of size dt = T/N
 * (Section 3.1), and for the compressed modes the cluster and block trees of
 * Section 4.1 (eq. qadm) with the Chebyshev bases of Section 4.2.
 *   vertices: host, nv x 3 doubles;  tris: host, M x 3 int32 vertex indices
 *   (0-based), both copied.  N >= 2 time steps on (0, T].  Triangles sharing
 *   a vertex index are the near field (singular quadrature of the Galerkin
 *   entries, Section 3.2).  Uploads per-mesh tables (library-owned, freed by
 *   cqm_problem_destroy).  opt may be NULL (defaults).
 *   CQM_EINVAL on degenerate triangles, out-of-range indices or bad options;
 *   CQM_EDEVICE if the upload fails. */
int cqm_problem_create(cqm_ctx_t ctx, const double* vertices, int64_t nv,
                       const int32_t* tris, int64_t M, int32_t N, double T,
                       const cqm_options* opt, cqm_problem_t* out);
int cqm_problem_destroy(cqm_problem_t p);

/* Bytes of device workspace a solve of this problem needs (host out).
 * Paper: no passage (memory plan; the storage it holds is that of
 * Section 6.2, Corollary cor:complex, for the compressed modes). */
int cqm_workspace_size(cqm_problem_t p, size_t* bytes);
/* Attach caller-owned device memory (>= cqm_workspace_size, 256-byte
 * aligned; the caller keeps ownership and must keep it alive while the
 * problem is used).  The library never allocates on the solve path.
 * CQM_ENOMEM if too small, CQM_EINVAL if NULL or misaligned.
 * Paper: no passage (memory plumbing). */
int cqm_set_workspace(cqm_problem_t p, void* dev_ptr, size_t bytes);

/* Incident data: the Dirichlet condition of Section 2.1 (eq. bc), projected
 * onto S_h^0 at every step t_n (the L2 projection of Section 3.2, with the
 * 6-point rule on each triangle).  Plane wave (host arguments):
 * g_D = -A exp(-((t - x.d - t0)/sigma)^2), d normalised by the library
 * (CQM_EINVAL for a zero direction or sigma <= 0).  Or caller samples of g_D
 * at the 6 quadrature points of every triangle: device, (N+1) x M x 6
 * doubles, caller-owned, read during cqm_solve (the pointer must stay
 * valid). */
int cqm_set_plane_wave(cqm_problem_t p, const double direction[3], double sigma,
                       double t0, double amplitude);
int cqm_set_dirichlet_samples(cqm_problem_t p, const double* g);

/* Solve the all-at-once form of the convolution quadrature (Section 3.1,
 * eq. cqm, omega_n, cqm_freq; the remark closing Section 6.2): right-hand
 * sides b_n (Section 3.2), the scaled transform ghat_l = sum_n rho^n b_n
 * zeta^-nl, one Galerkin system V(s_l) xhat_l = ghat_l per frequency, and
 * the inverse transform q_n = rho^-n/(N+1) sum_l xhat_l zeta^nl (eq. vhat,
 * eq. dft).  q_out: device, (N+1) x M doubles, caller-owned (density
 * coefficient of triangle i at step n).  diag: host, may be NULL.  Returns
 * CQM_ENOCONV (with output written) if some frequency missed outer_tol,
 * CQM_ENAN on non-finite data, CQM_ENOMEM without a workspace.  The call
 * waits for the stream: convergence is steered by flags the device writes
 * to host memory, so it returns after q_out is written. */
int cqm_solve(cqm_problem_t p, double* q_out, cqm_diag* diag, hipStream_t stream);

/* Solve `count` independent problems (different meshes, N and T allowed)
 * together, each as cqm_solve (Section 3.1, remark closing Section 6.2):
 * their frequency systems are batched in shared launches (batching itself
 * has no passage in the paper).
 * q_outs[k] and diags[k] as for cqm_solve (diags may be NULL).  The
 * problems must share gmres_restart, and those in the stored dense form
 * must share precond; otherwise CQM_EINVAL before any work is queued. */
int cqm_solve_batch(cqm_problem_t* probs, int32_t count, double** q_outs,
                    cqm_diag* diags, hipStream_t stream);

/* Time-marching solve of the same discrete system (Section 3.2, eq. dft,
 * eq. cqmgalapx with eq. cqmrhs): the real integration weights
 * What_n = rho^-n/(N+1) sum_l V(s_l) zeta^nl, n = 0..N, are formed from the
 * stored operator of the distinct frequencies, then for n = 0..N the history
 * sum r_n = b_n - sum_{j=1}^{n} What_j q_{n-j} and What_0 q_n = r_n (real
 * symmetric positive definite; conjugate gradients with the inverses of its
 * 64 x 64 diagonal blocks, to outer_tol relative residual).  It agrees with
 * cqm_solve up to terms of order rho^(N+1).  The problem must be created
 * with cqm_options.marching = 1 and the indirect formulation, either in a
 * plain mode with form CQM_FORM_DENSE, or in a compressed mode (Section 6.2:
 * the weights are the compressed operator with its fibres transformed,
 * eq. fastdft; the history sums use eq. fastrhs; needs aca_band
 * CQM_BAND_FULL and precond CQM_PRECOND_BLOCK_JACOBI); CQM_EINVAL
 * otherwise.  q_out: device, (N+1) x M doubles, caller-owned,
 * written step by step.  diag (host, may be NULL): total_iters / max_iters
 * are conjugate-gradient iterations over / per step, max_rel_residual the
 * largest final relative residual of a step.  CQM_ENOCONV if a step missed
 * its tolerance (output written), CQM_ENAN on non-finite values.  The call
 * waits for the stream (the host steers the iterations). */
int cqm_solve_marching(cqm_problem_t p, double* q_out, cqm_diag* diag, hipStream_t stream);

/* ------------------------------------------------------------ test hooks */
/* BDF2 CQM frequencies s_l = delta(rho zeta^-l)/dt for N steps on (0,T]
 * (Section 3.1, eq. cqm_freq; delta(xi) = (1-xi)(3-xi)/2); rho = 0 selects
 * rho^N = 1e-8.
 * s_re, s_im: host arrays of N+1 doubles.  CQM_EINVAL unless N >= 1, T > 0
 * and 0 <= rho < 1. */
int cqm_frequencies(int32_t N, double T, double rho, double* s_re, double* s_im);

/* y_l = V(s_l) x_l for l = l0 .. l0+nl-1: the Galerkin matrices
 * V_l[m,i] = <phi_m, V(s_l) phi_i> of Section 3.2 with the kernel of
 * eq. fundsol (plain modes), or their compressed form of Section 6,
 * eq. lrfinal (H2 x MACA modes), in the given precision (32 or 64; 32 is the
 * inner-iteration operator).  x, y: device complex arrays nl x M
 * (caller-owned, triangle order of the caller).  Assembles what the operator
 * needs on first use, into the workspace.  CQM_EINVAL for a frequency range
 * outside the solved band or a bad precision; CQM_ENOMEM without a
 * workspace. */
int cqm_apply_V(cqm_problem_t p, int32_t l0, int32_t nl, int32_t precision,
                const void* x, void* y, hipStream_t stream);

/* y_l = K(s_l) x_l for l = l0 .. l0+nl-1: the piecewise-constant Galerkin
 * matrices of the double-layer operator of Section 2.2 (eq. wavebio),
 * K_l[m,i] = <phi_m, K(s_l) phi_i>, kernel d/dn_y exp(-s r)/(4 pi r) with
 * n_y the unit normal of the source triangle in its vertex order; with
 * adjoint != 0 the adjoint double layer K' of the same equation (kernel
 * d/dn_x, the target's normal; for piecewise constants its matrix is K's
 * transpose).  FP64, far field matrix-free.  x, y: device complex128
 * arrays nl x M (caller-owned, must not overlap).  Needs a problem created
 * with formulation = CQM_FORMULATION_DIRECT (the workspace holds K's near
 * values and partial sums), else CQM_EINVAL; CQM_EINVAL for a frequency
 * range outside the solved band; CQM_ENOMEM without a workspace. */
int cqm_apply_K(cqm_problem_t p, int32_t l0, int32_t nl, int32_t adjoint, const void* x, void* y,
                hipStream_t stream);

/* y_l = D(s_l) x_l for l = l0 .. l0+nl-1: the Galerkin matrices of the
 * hypersingular operator of Section 2.2 (eq. wavebio) on the continuous
 * piecewise-linear space S_h^1 of Section 3.2, D_l[p,j] = <phi_p, D(s_l) phi_j>
 * over the hat functions of the mesh vertices.  The entries are those of the
 * integration by parts on the closed surface,
 *   int int G [curl phi_j(y) . curl phi_p(x) + s^2 n_x.n_y phi_j(y) phi_p(x)],
 * G = exp(-s r)/(4 pi r), the sign with which D_l is elliptic (Section 3.1);
 * pairs of triangles sharing a vertex take the static part 1/(4 pi r) by
 * Sauter-Schwab quadrature (q_duffy points per axis), once per mesh, the
 * rest by the 6-point rule; the far field matrix-free.  FP64.
 * x, y: device complex128 arrays nl x nv (vertex order of the mesh given to
 * cqm_problem_create; caller-owned, must not overlap).  Needs a problem
 * created with formulation = CQM_FORMULATION_DIRECT (the workspace holds the
 * product's per-triangle sources and partial sums), else CQM_EINVAL;
 * CQM_EINVAL for a frequency range outside the solved band; CQM_ENOMEM
 * without a workspace. */
int cqm_apply_D(cqm_problem_t p, int32_t l0, int32_t nl, const void* x, void* y, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): cqm_apply_V of the matrix-free
 * plain form (CQM_FORM_MATRIX_FREE, plain modes) with no allocation.  The
 * far product's split-K partial sums go to a fixed device array of 64 MiB
 * inside the library (one per GPU, held until the process ends); near-field
 * values go to the caller's workspace as in cqm_apply_V.  No hipMalloc,
 * hipFree or allocating call is made (no autotuning: the cached tuned shape
 * or the default one, its source split reduced to fit).  Arguments as for
 * cqm_apply_V.  CQM_EINVAL for other forms; CQM_ENOMEM when
 * nl x M x (8 or 16 bytes) exceeds 64 MiB, or without a workspace.  Every
 * call on one GPU shares that array and leaves its partial sums there:
 * calls that overlap on one GPU (other streams or threads) race. */
int cqm_apply_V_noalloc(cqm_problem_t p, int32_t l0, int32_t nl, int32_t precision,
                        const void* x, void* y, hipStream_t stream);

/* Near-field (vertex-sharing) pairs and their static Duffy integrals: the
 * singular part of the Galerkin entries of Section 3.2 (kernel of
 * eq. fundsol at s = 0).  Host arrays, caller-owned; pass NULL to query
 * *nnz first.  row_ptr: M+1, col: nnz, static_vals: nnz doubles (integral
 * of 1/(4 pi |x-y|) over the pair).  CQM_EINVAL on NULL p or nnz. */
int cqm_near_entries(cqm_problem_t p, int64_t* nnz, int32_t* row_ptr,
                     int32_t* col, double* static_vals);

/* Operator statistics after a solve or apply (host struct; solve fields 0):
 * block counts of the partition (Section 4.1), MACA ranks (Section 5.1,
 * Algorithm 2) and the operator's storage (Section 6.2, Corollary
 * cor:complex).  CQM_EINVAL on NULL arguments. */
int cqm_operator_stats(cqm_problem_t p, cqm_diag* out);

/* ------------------------------------------------------------ serving */
/* A server admits solve requests as they arrive, keeps every admitted
 * request's frequency-system states on the device and advances all of them
 * together, one GMRES restart cycle at a time; requests join and leave at
 * cycle boundaries (continuous batching).  Device memory comes from one arena
 * of hbm_budget bytes allocated at creation: a request is admitted when its
 * state (and, on a cache miss, its operator) fits, otherwise it waits; a
 * request that can never fit is rejected with CQM_ENOMEM.  Requests with the
 * same mesh, N and T share one operator (operator cache). */
typedef struct cqm_server_opts {
  int32_t max_active;      /* requests advanced together per lane        (16) */
  int32_t cache_operators; /* share operators of identical mesh, N, T     (1) */
  int32_t large_lane;      /* nonzero: requests whose stored dense operator
                              (plain form) would exceed large_bytes are
                              solved in the compressed form (H2 x MACA) by a
                              second worker on its own stream             (0) */
  int32_t fail_after_cycles; /* failure-path test hook: > 0 makes lane 0's
                              worker stop with CQM_EDEVICE after that many
                              restart cycles, as after a device error     (0) */
  int32_t large_cu_percent; /* share of the compute units the large lane's
                              stream may use (a CU mask spread evenly over
                              the chip), so the first lane always keeps the
                              rest; 0 or >= 100: no mask.  If the runtime
                              refuses the mask the stream is unmasked   (50) */
  int32_t reserved[3];
  int64_t large_bytes;     /* size limit of the above; <= 0: budget / 4   (0) */
  cqm_options solver;      /* options of every request (mode, form, tolerances) */
} cqm_server_opts;

typedef struct cqm_request {
  const double* vertices;  /* host, nv x 3 (copied at submit) */
  int64_t nv;
  const int32_t* tris;     /* host, M x 3 (copied at submit) */
  int64_t M;
  int32_t N;
  double T;
  double direction[3];     /* plane wave g_D = -A exp(-((t - x.d - t0)/sigma)^2) */
  double sigma, t0, amplitude;
} cqm_request;

typedef struct cqm_server_stats {
  int64_t submitted, completed, rejected, active, queued, peak_active;
  int64_t arena_bytes, peak_arena_bytes, operators_built, operator_cache_hits, cycles;
  int64_t lane_completed[2]; /* completed requests per lane (1: large)    */
  int64_t arena_used;        /* arena bytes held now (states + operators) */
  int64_t reserved[2];
} cqm_server_stats_t;

/* Default server options (host).  Paper: no passage (serving loop). */
int cqm_server_default_options(cqm_server_opts* opts);
/* Start a server on ctx's device with an arena of hbm_budget bytes
 * (library-owned until cqm_server_destroy).  CQM_ENOMEM if the arena cannot
 * be allocated.  Paper: no passage (serving loop). */
int cqm_server_create(cqm_ctx_t ctx, size_t hbm_budget, const cqm_server_opts* opts,
                      cqm_server_t* out);
/* Queue a request (mesh copied); *ticket identifies it.  Returns at once.
 * Each request is solved as cqm_solve (Section 3.1, remark closing
 * Section 6.2).  CQM_EINVAL on bad arguments; CQM_EDEVICE (nothing queued)
 * when the lane the request belongs to has stopped after a device error. */
int cqm_server_submit(cqm_server_t s, const cqm_request* req, uint64_t* ticket);
/* Paper: no passage (serving loop).
 * *done: 0 queued or running, 1 finished (return value: the request's
 * CQM_OK / CQM_ENOCONV / CQM_ENAN), -1 rejected (return value CQM_ENOMEM or
 * CQM_EINVAL).  When finished, q_out (host, (N+1) x M doubles, may be NULL),
 * diag (may be NULL) and latency_ms (submit to completion, may be NULL) are
 * written.  A finished ticket stays readable until the server is destroyed. */
int cqm_server_poll(cqm_server_t s, uint64_t ticket, int32_t* done, double* q_out,
                    cqm_diag* diag, double* latency_ms);
/* Block until every submitted request has finished or been rejected.
 * CQM_EDEVICE if a lane stopped after a device error (its requests are
 * rejected with CQM_EDEVICE).  Paper: no passage (serving loop). */
int cqm_server_drain(cqm_server_t s);
/* Counters of the server (host struct).  Paper: no passage. */
int cqm_server_stats(cqm_server_t s, cqm_server_stats_t* out);
/* Drain, stop the worker and release the arena.  Paper: no passage. */
int cqm_server_destroy(cqm_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* CQM_H */
