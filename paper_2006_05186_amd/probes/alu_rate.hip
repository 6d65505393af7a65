// Throughput probe of the vector ALU on the current device: lane operations
// per second of single instructions that the far-field kernels lean on
// (v_exp_f32, v_sin_f32, v_cos_f32, v_rsq_f32, FP32 FMA, FP64 FMA).  Each
// thread runs kChains independent dependency chains of one instruction so the
// issue rate, not the latency, bounds the loop.  Built as its own small
// library (not part of the C ABI of libcqm.so); bench.py --alu-probe calls it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {
constexpr int kChains = 8;
constexpr int kThreads = 256;

enum Op { kExp = 0, kSin, kCos, kRsq, kFma32, kFma64, kOps };

template <int OP>
__global__ __launch_bounds__(kThreads) void k_rate(const float* __restrict__ seed, int iters,
                                                   float* __restrict__ out) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  float x[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = seed[c] + 1e-3f * (float)(threadIdx.x & 7);
    d[c] = (double)x[c];
  }
  const float a = seed[kChains], b = seed[kChains + 1];
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == kExp) x[c] = __builtin_amdgcn_exp2f(-x[c]);       // fixed point ~0.64
      if constexpr (OP == kSin) x[c] = __builtin_amdgcn_sinf(x[c]);         // revolutions
      if constexpr (OP == kCos) x[c] = __builtin_amdgcn_cosf(x[c]);
      if constexpr (OP == kRsq) x[c] = __builtin_amdgcn_rsqf(x[c]);         // x > 0 stays > 0
      if constexpr (OP == kFma32) x[c] = __builtin_fmaf(x[c], a, b);
      if constexpr (OP == kFma64) d[c] = __builtin_fma(d[c], (double)a, (double)b);
    }
  }
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += x[c] + (float)d[c];
  out[t] = acc;
}

template <int OP>
float time_op(int blocks, int iters, const float* seed, float* out, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(kThreads), 0, s, seed, iters, out);  // warm-up
  hipEventRecord(e0, s);
  hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(kThreads), 0, s, seed, iters, out);
  hipEventRecord(e1, s);
  float ms = -1.f;
  if (hipEventSynchronize(e1) == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}
}  // namespace

extern "C" {
// rates[6]: lane operations per second of exp, sin, cos, rsq, FP32 FMA and
// FP64 FMA on device `device`, `blocks` workgroups of 256 threads, `iters`
// iterations of 8 chains each.  Returns 0, or -1 on a HIP error.
int cqm_probe_alu_rates(int device, int blocks, int iters, double* rates) {
  if (blocks < 1 || iters < 1 || !rates || hipSetDevice(device) != hipSuccess) return -1;
  float* seed = nullptr;
  float* out = nullptr;
  const float h_seed[kChains + 2] = {0.11f, 0.23f, 0.37f, 0.41f, 0.53f, 0.67f, 0.71f, 0.83f,
                                     0.999f, 1e-4f};
  if (hipMalloc(&seed, sizeof(h_seed)) != hipSuccess) return -1;
  if (hipMalloc(&out, sizeof(float) * (size_t)blocks * kThreads) != hipSuccess) {
    hipFree(seed);
    return -1;
  }
  int rc = hipMemcpy(seed, h_seed, sizeof(h_seed), hipMemcpyHostToDevice) == hipSuccess ? 0 : -1;
  const double lane_ops = (double)blocks * kThreads * iters * kChains;
  float ms[kOps];
  if (rc == 0) {
    ms[kExp] = time_op<kExp>(blocks, iters, seed, out, nullptr);
    ms[kSin] = time_op<kSin>(blocks, iters, seed, out, nullptr);
    ms[kCos] = time_op<kCos>(blocks, iters, seed, out, nullptr);
    ms[kRsq] = time_op<kRsq>(blocks, iters, seed, out, nullptr);
    ms[kFma32] = time_op<kFma32>(blocks, iters, seed, out, nullptr);
    ms[kFma64] = time_op<kFma64>(blocks, iters, seed, out, nullptr);
    for (int k = 0; k < kOps; ++k) {
      if (!(ms[k] > 0.f)) rc = -1;
      rates[k] = ms[k] > 0.f ? lane_ops / (ms[k] * 1e-3) : 0.0;
    }
  }
  hipFree(seed);
  hipFree(out);
  return rc;
}
}
