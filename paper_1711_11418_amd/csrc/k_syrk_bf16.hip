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
  if (I.sb) return;   // built by the direct-to-LDS kernel
  const int nt = (int)ceil_div<int64_t>(I.np, kT);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= I.ksplit) return;
  int ti, tj;
  tile_index(blockIdx.x, nt, ti, tj);
  const int64_t ld = I.split_ld, np = I.np, rows = I.rows;
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

// Wide parameter sets: direct-to-LDS staged tiles of side T = 64 B.  One
// workgroup of four wavefronts owns a T x T tile of the upper triangle; each
// wavefront accumulates a (T/2) x (T/2) quadrant as B x B blocks of 32 x 32
// MFMA accumulators.  The contraction runs in steps of 16 samples (two
// groups of 8).  A step's operands, the hi and lo halves of both T-parameter
// ranges, go straight from global memory into one of four LDS stages
// (global_load_lds, no staging registers), issued three steps ahead and
// interleaved one per MFMA; a step's operands are read from LDS into
// registers one step ahead, interleaved the same way.  One barrier per step
// publishes the next stage.  The split arrays are padded (parameters to
// split_ld, samples to a multiple of 32) so no load is guarded.
//
// Tiles past the last full round of the GPU are split over the samples
// (tail_ks parts); their FP32 partial tiles are summed in part order by
// k_syrk_tail, so S is deterministic.  Whole tiles write S directly.
namespace {
template <int B>
struct Ops {
  bf16x8 ah[B], al[B], bh[B], bl[B];
};
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gbl_void_t;

template <int B>
struct DmaTile {
  static constexpr int T = 64 * B;
  static constexpr int V = 8 * T;          // 16-byte vectors per stage: [hiA|loA|hiB|loB][2 groups][T]
  static constexpr int PT = V / 256;       // vectors per thread and stage
  static constexpr int kStages = 4;
};

// Steps [s0, s1) (both even) of the tile at (p0, q0); writes S (part null)
// or the unscaled FP32 partial tile.
template <int B>
__device__ __forceinline__ void syrk_dma_tile(const uint16_t* __restrict__ hi, int64_t lo_elems,
                                              int64_t sld, int64_t np, float invN,
                                              float* __restrict__ S, int64_t p0, int64_t q0,
                                              bool diag, u16x8* stage, int64_t s0, int64_t s1,
                                              float* __restrict__ part) {
  using C = DmaTile<B>;
  constexpr int T = C::T, V = C::V, PT = C::PT, H = T / 2;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, m = lane & 31, kh = lane >> 5;
  const int qi = wv >> 1, qj = wv & 1;
  // byte offset of each of this thread's vectors from the step's hi base
  uint32_t off[PT];
#pragma unroll
  for (int e = 0; e < PT; ++e) {
    const int v = tid + 256 * e;
    const int arr = v / (2 * T), g = (v / T) % 2, p = v % T;
    const int64_t col = (arr < 2 ? p0 : q0) + p;
    off[e] = (uint32_t)(((arr & 1) ? lo_elems * 2 : 0) + ((int64_t)g * sld + col) * 16);
  }
  auto dma = [&](int64_t s, int st) {
    const char* base = reinterpret_cast<const char*>(hi) + s * 2 * sld * 16;
#pragma unroll
    for (int e = 0; e < PT; ++e)
      __builtin_amdgcn_global_load_lds((gbl_void_t*)(base + off[e]),
                                       (lds_void_t*)(stage + st * V + 256 * e + 64 * wv), 16, 0, 0);
  };
  auto lread = [&](Ops<B>& o, int st) {
    const u16x8* sp = stage + st * V + kh * T;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int pa = H * qi + 32 * i + m, pb = H * qj + 32 * i + m;
      o.ah[i] = __builtin_bit_cast(bf16x8, sp[pa]);
      o.al[i] = __builtin_bit_cast(bf16x8, sp[2 * T + pa]);
      o.bh[i] = __builtin_bit_cast(bf16x8, sp[4 * T + pb]);
      o.bl[i] = __builtin_bit_cast(bf16x8, sp[6 * T + pb]);
    }
  };
  f32x16 acc[B][B];
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  auto pass = [&](const bf16x8 (&a)[B], const bf16x8 (&b)[B]) {
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int j = 0; j < B; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  // s_waitcnt with vmcnt <= 2 PT (the two later steps stay in flight)
  constexpr int W2 = 2 * PT;
  constexpr int kWait2 = (W2 & 15) | ((W2 >> 4) << 14) | (7 << 4) | (15 << 8);
  const int64_t last = s1 - 1;
  // One step: issue the loads of step s + 3 among the first pass of
  // products, wait for step s + 1 and publish it, then read its operands
  // among the remaining two passes.
  auto step = [&](int64_t s, Ops<B>& X, Ops<B>& Y) {
    dma(s + 3 <= last ? s + 3 : last, (int)((s + 3) & 3));
    pass(X.ah, X.bh);
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // one global load
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
    }
    __builtin_amdgcn_sched_group_barrier(0x008, B * B > PT ? B * B - PT : 0, 0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(kWait2);
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
    lread(Y, (int)((s + 1) & 3));
    pass(X.ah, X.bl);
    pass(X.al, X.bh);
#pragma unroll
    for (int k = 0; k < 4 * B; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 2 * B * B - 4 * B, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  dma(s0, (int)(s0 & 3));
  dma(s0 + 1 <= last ? s0 + 1 : last, (int)((s0 + 1) & 3));
  dma(s0 + 2 <= last ? s0 + 2 : last, (int)((s0 + 2) & 3));
  __builtin_amdgcn_s_waitcnt(kWait2);
  __builtin_amdgcn_s_barrier();
  Ops<B> X, Y;
  lread(X, (int)(s0 & 3));
  for (int64_t s = s0; s < s1; s += 2) {
    step(s, X, Y);
    step(s + 1, Y, X);
  }
  // no load may still be writing this workgroup's LDS when it exits
  __builtin_amdgcn_s_waitcnt(0);
  // accumulator r of lane l holds D[row][col], col = l % 32,
  // row = 8 (r / 4) + 4 (l / 32) + r % 4
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int lr = H * qi + 32 * i + 8 * (r >> 2) + 4 * kh + (r & 3);
        const int lc = H * qj + 32 * j + m;
        if (part) {
          part[lr * T + lc] = acc[i][j][r];
        } else {
          const int64_t row = p0 + lr, col = q0 + lc;
          if (row < np && col < np && (!diag || row <= col)) {
            const float v = acc[i][j][r] * invN;
            S[row * np + col] = v;
            S[col * np + row] = v;
          }
        }
      }
}

// unit u of an instance: a whole tile (u < nfull) or part k of tail tile t
__device__ __forceinline__ void unit_of(int u, int nfull, int ks, int& t, int& k) {
  if (u < nfull) {
    t = u;
    k = -1;
  } else {
    t = nfull + (u - nfull) / ks;
    k = (u - nfull) % ks;
  }
}
}  // namespace

template <int B>
__global__ __launch_bounds__(256) void k_syrk_dma(SrArgs A, const uint16_t* __restrict__ split,
                                                  float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (I.sb != B) return;
  constexpr int T = DmaTile<B>::T;
  const int nt = (int)ceil_div<int64_t>(I.np, T);
  const int ntl = nt * (nt + 1) / 2;
  const int nunits = I.nfull + (ntl - I.nfull) * I.tail_ks;
  if ((int)blockIdx.x >= nunits) return;
  __shared__ u16x8 stage[DmaTile<B>::kStages * DmaTile<B>::V];
  int t, k;
  unit_of(blockIdx.x, I.nfull, I.tail_ks, t, k);
  int ti, tj;
  tile_index(t, nt, ti, tj);
  const int64_t steps = (I.rows + 31) / 32 * 2;   // 16-sample steps, an even count
  int64_t s0 = 0, s1 = steps;
  float* part = nullptr;
  if (k >= 0) {
    const int64_t chunk = ceil_div<int64_t>(steps / 2, I.tail_ks) * 2;
    s0 = k * chunk;
    s1 = s0 + chunk < steps ? s0 + chunk : steps;
    part = reinterpret_cast<float*>(A.syrkpart + I.syrkpart_off) +
           ((int64_t)(t - I.nfull) * I.tail_ks + k) * T * T;
    if (s0 >= s1) {   // empty part: contributes zero
      for (int e = threadIdx.x; e < T * T; e += blockDim.x) part[e] = 0.f;
      return;
    }
  }
  const uint16_t* hi = split + I.split_off;
  const float invN = (float)(1.0 / (double)I.rows);
  syrk_dma_tile<B>(hi, I.split_rows * I.split_ld, I.split_ld, I.np, invN, S + I.S_off,
                   (int64_t)ti * T, (int64_t)tj * T, ti == tj, stage, s0, s1, part);
}

// Tail tiles: sum the sample parts in order, scale by 1/N, write both triangles.
template <int B>
__global__ void k_syrk_tail(SrArgs A, float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.z];
  if (I.sb != B) return;
  constexpr int T = DmaTile<B>::T;
  const int nt = (int)ceil_div<int64_t>(I.np, T);
  const int ntl = nt * (nt + 1) / 2;
  const int tt = I.nfull + (int)blockIdx.y;
  if (tt >= ntl) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= T * T) return;
  int ti, tj;
  tile_index(tt, nt, ti, tj);
  const int lr = e / T, lc = e % T;
  const int64_t row = (int64_t)ti * T + lr, col = (int64_t)tj * T + lc;
  if (row >= I.np || col >= I.np || (ti == tj && row > col)) return;
  const float* part = reinterpret_cast<const float*>(A.syrkpart + I.syrkpart_off) +
                      (int64_t)blockIdx.y * I.tail_ks * T * T;
  float a = 0.f;
  for (int k = 0; k < I.tail_ks; ++k) a += part[(int64_t)k * T * T + e];
  const float v = a * (float)(1.0 / (double)I.rows);
  float* Sb = S + I.S_off;
  Sb[row * I.np + col] = v;
  Sb[col * I.np + row] = v;
}

__global__ void k_syrk_split_reduce(SrArgs A, float* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (I.sb || I.ksplit == 1) return;   // written directly by a tile kernel
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
                    int max_ksplit, const SyrkLaunch& L, hipStream_t s) {
  if (L.any64) {
    const int nt = (int)ceil_div<int64_t>(max_np, kT);
    const int ntiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(k_syrk_mfma, dim3(ntiles, max_ksplit, n_inst), dim3(64), 0, s, A, split, S);
    if (max_ksplit > 1)
      hipLaunchKernelGGL(k_syrk_split_reduce, dim3(ntiles, n_inst), dim3(256), 0, s, A, S);
  }
  if (L.units[2]) {
    hipLaunchKernelGGL(k_syrk_dma<2>, dim3(L.units[2], n_inst), dim3(256), 0, s, A, split, S);
    if (L.tail[2])
      hipLaunchKernelGGL(k_syrk_tail<2>, dim3(128 * 128 / 256, L.tail[2], n_inst), dim3(256), 0, s, A, S);
  }
  if (L.units[3]) {
    hipLaunchKernelGGL(k_syrk_dma<3>, dim3(L.units[3], n_inst), dim3(256), 0, s, A, split, S);
    if (L.tail[3])
      hipLaunchKernelGGL(k_syrk_tail<3>, dim3(192 * 192 / 256, L.tail[3], n_inst), dim3(256), 0, s, A, S);
  }
  if (L.units[4]) {
    hipLaunchKernelGGL(k_syrk_dma<4>, dim3(L.units[4], n_inst), dim3(256), 0, s, A, split, S);
    if (L.tail[4])
      hipLaunchKernelGGL(k_syrk_tail<4>, dim3(256 * 256 / 256, L.tail[4], n_inst), dim3(256), 0, s, A, S);
  }
}

}  // namespace mvmc
