// Split-bf16 S build on the matrix cores (gfx950 v_mfma_f32_32x32x16_bf16).
//
// The centred single-precision O~ is stored as hi = bf16(O~) and
// lo = bf16(O~ - hi) in a k-blocked layout (split_index in sr.h); S = O~^T O~ / N
// is accumulated in FP32 as hi^T hi + hi^T lo + lo^T hi (the lo^T lo term is
// below single-precision resolution).  One wavefront computes a 64 x 64 tile
// of the upper triangle as 2 x 2 blocks of 32 x 32 MFMA accumulators; the
// contraction runs over the samples, 16 per MFMA.
#include "sr.h"

namespace mvmc {

namespace {
constexpr int kT = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void tile_index(int t, int nt, int& ti, int& tj) {
  int row = 0, start = 0;
  while (t >= start + (nt - row)) {
    start += nt - row;
    ++row;
  }
  ti = row;
  tj = row + (t - start);
}

// Eight consecutive samples of one parameter (zero beyond the used rows).
__device__ __forceinline__ bf16x8 load8(const uint16_t* __restrict__ base, int64_t kg, int64_t p,
                                        int64_t ld, bool ok, int valid) {
  u16x8 v = {0, 0, 0, 0, 0, 0, 0, 0};
  if (ok) {
    v = *reinterpret_cast<const u16x8*>(base + (kg * ld + p) * 8);
    if (valid < 8) {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (e >= valid) v[e] = 0;
    }
  }
  return __builtin_bit_cast(bf16x8, v);
}
}  // namespace

__global__ __launch_bounds__(64) void k_syrk_mfma(SrArgs A, const uint16_t* __restrict__ split,
                                                  float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.z];
  if (I.tile128) return;   // built by the 128-tile kernel
  const int nt = (int)ceil_div<int64_t>(I.np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= I.ksplit) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const int64_t ld = I.ldO, np = I.np, rows = I.rows;
  const int64_t chunk = ceil_div<int64_t>(ceil_div<int64_t>(rows, I.ksplit), 16) * 16;
  const int64_t k0 = (int64_t)blockIdx.y * chunk;
  const int64_t k1 = k0 + chunk < rows ? k0 + chunk : rows;
  const uint16_t* hi = split + I.split_off;
  const uint16_t* lo = hi + I.split_rows * ld;
  const int lane = threadIdx.x, m = lane & 31, kh = lane >> 5;
  const int64_t p0 = (int64_t)ti * kT, q0 = (int64_t)tj * kT;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  for (int64_t k = k0; k < k1; k += 16) {
    const int64_t kg = (k >> 3) + kh;                 // this lane's group of 8 samples
    const int64_t left = rows - kg * 8;
    const int valid = left >= 8 ? 8 : (left > 0 ? (int)left : 0);
    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int64_t p = p0 + 32 * i + m, q = q0 + 32 * i + m;
      ah[i] = load8(hi, kg, p, ld, p < np && valid > 0, valid);
      al[i] = load8(lo, kg, p, ld, p < np && valid > 0, valid);
      bh[i] = load8(hi, kg, q, ld, q < np && valid > 0, valid);
      bl[i] = load8(lo, kg, q, ld, q < np && valid > 0, valid);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
  // accumulator r of lane l holds D[row][col], col = l % 32,
  // row = 8 (r / 4) + 4 (l / 32) + r % 4
  const bool direct = I.ksplit == 1;
  const float invN = (float)(1.0 / (double)rows);
  double* part = A.syrkpart + I.syrkpart_off + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * kT * kT;
  float* Sb = S + I.S_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int lr = 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int lc = 32 * j + m;
        const float v = acc[i][j][r];
        if (direct) {
          const int64_t row = p0 + lr, col = q0 + lc;
          if (row < np && col < np && (ti != tj || row <= col)) {
            Sb[row * np + col] = v * invN;
            Sb[col * np + row] = v * invN;
          }
        } else {
          part[lr * kT + lc] = (double)v;
        }
      }
}

// Wide parameter sets: one wavefront per 128 x 128 tile of the upper
// triangle, 4 x 4 blocks of 32 x 32 accumulators (held in the accumulation
// registers), three bf16 products per block and 16 samples, so each
// 16-sample step loads 16 operand vectors for 48 MFMAs (three times the
// operand reuse of the 64-tile kernel).  The next step's operands are loaded
// before the current step's products are issued.  No K split: S is written
// directly, both triangles.
namespace {
constexpr int kT2 = 128;
struct Ops128 {
  bf16x8 ah[4], al[4], bh[4], bl[4];
};
// Operands of one 16-sample step.  The split arrays hold zeros up to the
// next multiple of 16 samples and in the padding parameters (rows of O are
// padded to a multiple of 128 for these instances), so no load is masked.
__device__ __forceinline__ bf16x8 load8u(const uint16_t* __restrict__ p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(p));
}
__device__ __forceinline__ void load_ops128(Ops128& o, const uint16_t* hi, const uint16_t* lo,
                                            int64_t k, int64_t ld, int64_t p0, int64_t q0,
                                            int m, int kh) {
  const int64_t kg = (k >> 3) + kh;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t ip = (kg * ld + p0 + 32 * i + m) * 8, iq = (kg * ld + q0 + 32 * i + m) * 8;
    o.ah[i] = load8u(hi + ip);
    o.al[i] = load8u(lo + ip);
    o.bh[i] = load8u(hi + iq);
    o.bl[i] = load8u(lo + iq);
  }
}
__device__ __forceinline__ void mfma_step128(f32x16 (&acc)[4][4], const Ops128& o) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[i], o.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[i], o.bh[j], acc[i][j], 0, 0, 0);
}
}  // namespace

__global__ __launch_bounds__(64) void k_syrk_mfma128(SrArgs A, const uint16_t* __restrict__ split,
                                                     float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (!I.tile128) return;
  const int nt = (int)ceil_div<int64_t>(I.np, kT2);
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const int64_t ld = I.ldO, np = I.np, rows = I.rows;
  const uint16_t* hi = split + I.split_off;
  const uint16_t* lo = hi + I.split_rows * ld;
  const int lane = threadIdx.x, m = lane & 31, kh = lane >> 5;
  const int64_t p0 = (int64_t)ti * kT2, q0 = (int64_t)tj * kT2;
  f32x16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // The products run pass by pass, so each accumulator's dependent MFMAs
  // are 16 issues apart; the loads of a step are unconditional (the last
  // step reloads itself), which keeps the number in flight fixed.
  Ops128 cur, nxt;
  const int64_t rows16 = (rows + 15) / 16 * 16;
  load_ops128(cur, hi, lo, 0, ld, p0, q0, m, kh);
  for (int64_t k = 0; k < rows16; k += 16) {
    load_ops128(nxt, hi, lo, k + 16 < rows16 ? k + 16 : k, ld, p0, q0, m, kh);
    mfma_step128(acc, cur);
    cur = nxt;
  }
  // accumulator r of lane l holds D[row][col], col = l % 32,
  // row = 8 (r / 4) + 4 (l / 32) + r % 4
  const float invN = (float)(1.0 / (double)rows);
  float* Sb = S + I.S_off;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = p0 + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int64_t col = q0 + 32 * j + m;
        if (row < np && col < np && (ti != tj || row <= col)) {
          const float v = acc[i][j][r] * invN;
          Sb[row * np + col] = v;
          Sb[col * np + row] = v;
        }
      }
}

// Wide parameter sets, LDS-staged: one workgroup of four wavefronts per
// 128 x 128 tile of the upper triangle, each wavefront a 64 x 64 quadrant
// (2 x 2 blocks of 32 x 32 accumulators).  Panels of 32 samples (four
// groups of 8) of the two 128-parameter ranges, hi and lo, pass from global
// memory through registers into one of two LDS buffers: the next panel's
// global loads are in flight while the current panel's products issue.
// Sample groups past the last multiple of 16 samples read as zero.
namespace {
constexpr int kStageVecs = 4 * 4 * 128;   // [hiA | loA | hiB | loB][group][parameter]
__device__ __forceinline__ void mfma_quad(f32x16 (&acc)[2][2], const bf16x8 (&ah)[2],
                                          const bf16x8 (&al)[2], const bf16x8 (&bh)[2],
                                          const bf16x8 (&bl)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
}
}  // namespace

__global__ __launch_bounds__(256) void k_syrk_lds128(SrArgs A, const uint16_t* __restrict__ split,
                                                     float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (!I.tile128) return;
  const int nt = (int)ceil_div<int64_t>(I.np, kT2);
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const int64_t ld = I.ldO, np = I.np, rows = I.rows;
  const int64_t ng = (rows + 15) / 16 * 2;   // groups of 8 samples in use
  const uint16_t* hi = split + I.split_off;
  const uint16_t* lo = hi + I.split_rows * ld;
  const int64_t p0 = (int64_t)ti * kT2, q0 = (int64_t)tj * kT2;
  __shared__ u16x8 stage[2][kStageVecs];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, m = lane & 31, kh = lane >> 5;
  const int qi = wv >> 1, qj = wv & 1;

  u16x8 reg[8];
  auto gload = [&](int64_t kg0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int v = tid + 256 * e;
      const int arr = v >> 9, g = (v >> 7) & 3, p = v & 127;
      const int64_t kg = kg0 + g;
      const int64_t col = (arr < 2 ? p0 : q0) + p;
      const uint16_t* base = (arr & 1) ? lo : hi;
      u16x8 z = {0, 0, 0, 0, 0, 0, 0, 0};
      reg[e] = kg < ng ? *reinterpret_cast<const u16x8*>(base + (kg * ld + col) * 8) : z;
    }
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int e = 0; e < 8; ++e) stage[b][tid + 256 * e] = reg[e];
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  gload(0);
  lstore(0);
  __syncthreads();
  int b = 0;
  for (int64_t kg0 = 0; kg0 < ng; kg0 += 4) {
    const bool more = kg0 + 4 < ng;
    if (more) gload(kg0 + 4);
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      const int g = 2 * sub + kh;
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int pa = g * 128 + 64 * qi + 32 * i + m, pb = g * 128 + 64 * qj + 32 * i + m;
        ah[i] = __builtin_bit_cast(bf16x8, stage[b][pa]);
        al[i] = __builtin_bit_cast(bf16x8, stage[b][512 + pa]);
        bh[i] = __builtin_bit_cast(bf16x8, stage[b][1024 + pb]);
        bl[i] = __builtin_bit_cast(bf16x8, stage[b][1536 + pb]);
      }
      mfma_quad(acc, ah, al, bh, bl);
    }
    if (more) lstore(b ^ 1);
    __syncthreads();
    b ^= 1;
  }
  // accumulator r of lane l holds D[row][col], col = l % 32,
  // row = 8 (r / 4) + 4 (l / 32) + r % 4
  const float invN = (float)(1.0 / (double)rows);
  float* Sb = S + I.S_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = p0 + 64 * qi + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int64_t col = q0 + 64 * qj + 32 * j + m;
        if (row < np && col < np && (ti != tj || row <= col)) {
          const float v = acc[i][j][r] * invN;
          Sb[row * np + col] = v;
          Sb[col * np + row] = v;
        }
      }
}

__global__ void k_syrk_split_reduce(SrArgs A, float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (I.ksplit == 1) return;   // written directly by the tile kernel
  const int nt = (int)ceil_div<int64_t>(I.np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const double* part = A.syrkpart + I.syrkpart_off;
  const double invN = 1.0 / (double)I.rows;
  float* Sb = S + I.S_off;
  for (int e = threadIdx.x; e < kT * kT; e += blockDim.x) {
    const int i = e / kT, j = e % kT;
    const int64_t r = (int64_t)ti * kT + i, c = (int64_t)tj * kT + j;
    if (r >= I.np || c >= I.np || (ti == tj && r > c)) continue;
    double s = 0.0;
    for (int ks = 0; ks < I.ksplit; ++ks) s += part[((int64_t)ks * ntiles + blockIdx.x) * kT * kT + e];
    const float v = (float)(s * invN);
    Sb[r * I.np + c] = v;
    Sb[c * I.np + r] = v;
  }
}

void sr_syrk_bf16x3(const SrArgs& A, const uint16_t* split, float* S, int n_inst, int64_t max_np,
                    int max_ksplit, hipStream_t s) {
  const int nt = (int)ceil_div<int64_t>(max_np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  hipLaunchKernelGGL(k_syrk_mfma, dim3(ntiles, max_ksplit, n_inst), dim3(64), 0, s, A, split, S);
  hipLaunchKernelGGL(k_syrk_split_reduce, dim3(ntiles, n_inst), dim3(256), 0, s, A, S);
  const int nt2 = (int)ceil_div<int64_t>(max_np, kT2);
  if (nt2 * (nt2 + 1) / 2 >= 512)
    hipLaunchKernelGGL(k_syrk_lds128, dim3(nt2 * (nt2 + 1) / 2, n_inst), dim3(256), 0, s, A,
                       split, S);
}

}  // namespace mvmc
