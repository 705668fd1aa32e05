// Attainable peaks for the roofline report: register-only loops of the
// instructions the hot path uses (bf16 MFMA 32x32x16, FP64 MFMA 16x16x4,
// FP64 vector FMA), on non-zero data, two wavefronts per SIMD.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace mvmc {

namespace {
typedef __bf16 p_bf16x8 __attribute__((ext_vector_type(8)));
typedef float p_f32x16 __attribute__((ext_vector_type(16)));
typedef double p_f64x4 __attribute__((ext_vector_type(4)));
constexpr int kProbeAcc = 8;   // independent accumulators per wavefront

__global__ __launch_bounds__(256) void k_probe_bf16(float* out, int iters) {
  p_f32x16 acc[kProbeAcc];
  for (int k = 0; k < kProbeAcc; ++k)
    for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
  p_bf16x8 a, b;
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(0.37f * (float)(threadIdx.x + e + 1));
    b[e] = (__bf16)(0.11f * (float)(3 * threadIdx.x + e + 1));
  }
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k)
      acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
  float s = 0.f;
  for (int k = 0; k < kProbeAcc; ++k)
    for (int r = 0; r < 16; ++r) s += acc[k][r];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_f64mfma(float* out, int iters) {
  p_f64x4 acc[kProbeAcc];
  for (int k = 0; k < kProbeAcc; ++k) acc[k] = p_f64x4{0.0, 0.0, 0.0, 0.0};
  const double a = 1e-3 * (threadIdx.x + 1), b = 3e-3 * (threadIdx.x + 7);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k)
      acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  double s = 0.0;
  for (int k = 0; k < kProbeAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

__global__ __launch_bounds__(256) void k_probe_f64fma(float* out, int iters) {
  double x[kProbeAcc];
  for (int k = 0; k < kProbeAcc; ++k) x[k] = 1e-3 * (threadIdx.x + k + 1);
  const double m = 0.999999, c = 1e-7;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int k = 0; k < kProbeAcc; ++k) x[k] = fma(x[k], m, c);
  double s = 0.0;
  for (int k = 0; k < kProbeAcc; ++k) s += x[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}
}  // namespace

// flops per wavefront and iteration of each probe
double probe_flops_per_wave_iter(int kind) {
  if (kind == 0) return kProbeAcc * 2.0 * 32 * 32 * 16;
  if (kind == 1) return kProbeAcc * 2.0 * 16 * 16 * 4;
  return kProbeAcc * 2.0 * 64;
}

void launch_probe(int kind, float* out, int blocks, int iters, hipStream_t s) {
  if (kind == 0) hipLaunchKernelGGL(k_probe_bf16, dim3(blocks), dim3(256), 0, s, out, iters);
  else if (kind == 1) hipLaunchKernelGGL(k_probe_f64mfma, dim3(blocks), dim3(256), 0, s, out, iters);
  else hipLaunchKernelGGL(k_probe_f64fma, dim3(blocks), dim3(256), 0, s, out, iters);
}

}  // namespace mvmc
