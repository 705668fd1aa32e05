// Split-bf16 S build for the mixed-precision path.
//
// The centred single-precision O~ is stored as hi = bf16(O~) and
// lo = bf16(O~ - hi); S = O~^T O~ / N is accumulated in FP32 as
// hi^T hi + hi^T lo + lo^T hi (the lo^T lo term is below FP32 resolution).
#include "sr.h"

namespace mvmc {

namespace {
constexpr int kT = 64, kK = 32;

__device__ __forceinline__ void tile_index(int t, int nt, int& ti, int& tj) {
  int row = 0, start = 0;
  while (t >= start + (nt - row)) {
    start += nt - row;
    ++row;
  }
  ti = row;
  tj = row + (t - start);
}
}  // namespace

__global__ __launch_bounds__(256) void k_syrk_split_vec(SrArgs A, const uint16_t* __restrict__ split) {
  const SrInst& I = A.inst[blockIdx.z];
  const int nt = (int)ceil_div<int64_t>(I.np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= I.ksplit) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const int64_t chunk = ceil_div<int64_t>(ceil_div<int64_t>(I.rows, I.ksplit), kK) * kK;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < I.rows ? r0 + chunk : I.rows;
  __shared__ float Ah[kK][kT + 1], Al[kK][kT + 1], Bh[kK][kT + 1], Bl[kK][kT + 1];
  const int64_t ld = I.ldO;
  const uint16_t* hi = split + I.split_off;
  const uint16_t* lo = hi + I.rows * ld;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  float acc[4][4] = {};
  const int ca = ti * kT, cb = tj * kT;
  for (int64_t m0 = r0; m0 < r1; m0 += kK) {
    for (int e = threadIdx.x; e < kK * kT; e += 256) {
      const int kk = e / kT, c = e % kT;
      const int64_t m = m0 + kk;
      const bool ok = m < r1;
      const bool oa = ok && ca + c < I.np, ob = ok && cb + c < I.np;
      Ah[kk][c] = oa ? bf16_to_f32(hi[m * ld + ca + c]) : 0.f;
      Al[kk][c] = oa ? bf16_to_f32(lo[m * ld + ca + c]) : 0.f;
      Bh[kk][c] = ob ? bf16_to_f32(hi[m * ld + cb + c]) : 0.f;
      Bl[kk][c] = ob ? bf16_to_f32(lo[m * ld + cb + c]) : 0.f;
    }
    __syncthreads();
    for (int kk = 0; kk < kK; ++kk) {
      float ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ah[i] = Ah[kk][ty * 4 + i];
        al[i] = Al[kk][ty * 4 + i];
        bh[i] = Bh[kk][tx * 4 + i];
        bl[i] = Bl[kk][tx * 4 + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += ah[i] * bh[j] + (ah[i] * bl[j] + al[i] * bh[j]);
    }
    __syncthreads();
  }
  double* part = A.syrkpart + I.syrkpart_off + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * kT * kT;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) part[(ty * 4 + i) * kT + tx * 4 + j] = (double)acc[i][j];
}

__global__ void k_syrk_split_reduce(SrArgs A, float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nt = (int)ceil_div<int64_t>(I.np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const double* part = A.syrkpart + I.syrkpart_off;
  const float invN = (float)(1.0 / (double)I.rows);
  float* Sb = S + I.S_off;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    const int64_t r = (int64_t)ti * kT + i, c = (int64_t)tj * kT + j;
    if (r >= I.np || c >= I.np) continue;
    float s = 0.f;
    for (int ks = 0; ks < I.ksplit; ++ks) s += (float)part[((int64_t)ks * ntiles + blockIdx.x) * kT * kT + e];
    s *= invN;
    Sb[r * I.np + c] = s;
    Sb[c * I.np + r] = s;
  }
}

void sr_syrk_bf16x3(const SrArgs& A, const uint16_t* split, float* S, int n_inst, int64_t max_np,
                    int max_ksplit, hipStream_t s) {
  const int nt = (int)ceil_div<int64_t>(max_np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_syrk_split_vec, dim3(ntiles, max_ksplit, n_inst), dim3(256), 0, s, A, split);
  hipLaunchKernelGGL(k_syrk_split_reduce, dim3(ntiles, n_inst), dim3(256), 0, s, A, S);
}

}  // namespace mvmc
