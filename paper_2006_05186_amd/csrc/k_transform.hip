// Right-hand side samples and the scaled DFTs between time steps and CQM
// frequencies (all FP64).
#include "device_util.h"

namespace cqm {

// b[n][i] = sum_a W_ia g_D(x_ia, t_n): L2 projection of the Dirichlet data
// onto piecewise constants with the 6-point rule (Section 3.2).
__global__ void k_rhs(const double4* __restrict__ pts, int M, int F, double dt, double dx,
                      double dy, double dz, double sigma, double t0, double amp,
                      const double* __restrict__ samples, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (i >= M || n >= F) return;
  const double t = n * dt;
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < kQ; ++a) {
    const double4 q = pts[i * kQ + a];
    double g;
    if (samples) {
      g = samples[((int64_t)n * M + i) * kQ + a];
    } else {
      const double u = (t - (q.x * dx + q.y * dy + q.z * dz) - t0) / sigma;
      g = -amp * exp(-u * u);
    }
    acc += q.w * g;
  }
  b[(int64_t)n * M + i] = acc;
}

void launch_rhs(const Problem& p, const Incident& inc, double* b, hipStream_t s) {
  dim3 grid((p.M + 255) / 256, p.F);
  const double* smp = inc.kind == 2 ? inc.samples : nullptr;
  hipLaunchKernelGGL(k_rhs, grid, dim3(256), 0, s, p.dev.pts64, (int)p.M, p.F, p.dt, inc.dir[0],
                     inc.dir[1], inc.dir[2], inc.sigma, inc.t0, inc.amp, smp, b);
  CQM_HIP(hipGetLastError());
}

// ghat[l][i] = sum_n rho^n b[n][i] zeta^-(n l mod F), l < nsys.  zero2: two
// accumulators of the inverse transform of the same solve, cleared here.
__global__ void k_dft_fwd(const double* __restrict__ b, const double* __restrict__ rho_pow,
                          const cf64* __restrict__ tw, int M, int F, cf64* __restrict__ ghat,
                          double* __restrict__ zero2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (zero2 && blockIdx.x == 0 && l == 0 && threadIdx.x < 2) zero2[threadIdx.x] = 0.0;
  if (i >= M) return;
  double re = 0.0, im = 0.0;
  int k = 0;  // (n * l) mod F, advanced incrementally
  for (int n = 0; n < F; ++n) {
    const double v = rho_pow[n] * b[(int64_t)n * M + i];
    const cf64 w = tw[k];
    re += v * w.re;
    im += v * w.im;
    k += l;
    if (k >= F) k -= F;
  }
  ghat[(int64_t)l * M + i] = cf64{re, im};
}

void launch_dft_forward(const Problem& p, const double* b, cf64* ghat, double* zero2,
                        hipStream_t s) {
  dim3 grid((p.M + 255) / 256, p.Fsys);
  hipLaunchKernelGGL(k_dft_fwd, grid, dim3(256), 0, s, b, p.dev.rho_pow, p.dev.tw_fwd, (int)p.M,
                     p.F, ghat, zero2);
  CQM_HIP(hipGetLastError());
}

// q[n][i] = Re[ rho^-n / F sum_l xhat_l zeta^(n l mod F) ].  Half band: the
// frequencies F-l are conjugates of l, so their terms equal those of l and the
// sum is real by construction.  Full band: the imaginary part is accumulated
// into *imag_sq (and the real part into *real_sq) as a symmetry check.
__global__ void k_dft_inv(const cf64* __restrict__ xhat, const double* __restrict__ rho_ipow,
                          const cf64* __restrict__ tw, int M, int F, int nsys, int full,
                          double* __restrict__ q, double* imag_sq, double* real_sq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  __shared__ double red[16];
  double re = 0.0, im = 0.0;
  if (i < M) {
    if (full) {
      int k = 0;
      for (int l = 0; l < F; ++l) {
        const cf64 x = xhat[(int64_t)l * M + i];
        const cf64 w = tw[k];
        re += x.re * w.re - x.im * w.im;
        im += x.re * w.im + x.im * w.re;
        k += n;
        if (k >= F) k -= F;
      }
    } else {
      re = xhat[i].re;
      const int pairs = (F - 1) / 2;
      int k = n % F;
      for (int l = 1; l <= pairs; ++l) {
        const cf64 x = xhat[(int64_t)l * M + i];
        const cf64 w = tw[k];
        re += 2.0 * (x.re * w.re - x.im * w.im);
        k += n;
        if (k >= F) k -= F;
      }
      if ((F & 1) == 0) {  // middle frequency l = F/2 is real-symmetric
        const int l = F / 2;
        const cf64 x = xhat[(int64_t)l * M + i];
        const cf64 w = tw[(int)(((int64_t)n * l) % F)];
        re += x.re * w.re - x.im * w.im;
      }
    }
    const double sc = rho_ipow[n];
    re *= sc;
    im *= sc;
    q[(int64_t)n * M + i] = re;
  }
  if (full && imag_sq) {
    const double a = block_sum(im * im, red);
    const double c = block_sum(re * re, red);
    if (threadIdx.x == 0) {
      atomicAdd(imag_sq, a);
      atomicAdd(real_sq, c);
    }
  }
}

void launch_dft_inverse(const Problem& p, const cf64* xhat, double* q, double* imag_sq,
                        double* real_sq, hipStream_t s) {
  dim3 grid((p.M + 255) / 256, p.F);
  hipLaunchKernelGGL(k_dft_inv, grid, dim3(256), 0, s, xhat, p.dev.rho_ipow, p.dev.tw_inv,
                     (int)p.M, p.F, p.Fsys, p.full_band() ? 1 : 0, q, imag_sq, real_sq);
  CQM_HIP(hipGetLastError());
}

// out[l] = ||v_l||_2 for nsys vectors of length M at stride `stride`.
__global__ void k_vec_norms(const cf64* __restrict__ v, int64_t stride, int M,
                            double* __restrict__ out) {
  __shared__ double red[16];
  const cf64* x = v + (int64_t)blockIdx.x * stride;
  double acc = 0.0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) acc += x[i].re * x[i].re + x[i].im * x[i].im;
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(acc);
}

void launch_vec_norms(const cf64* v, int64_t stride, int M, int nsys, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_norms, dim3(nsys), dim3(256), 0, s, v, stride, M, out);
  CQM_HIP(hipGetLastError());
}

}  // namespace cqm
