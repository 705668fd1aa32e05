// Stochastic reconfiguration on the GPU (section 3.3.1, Eq. SR_equation_system;
// section 3.3.2, Algorithm 1).
//
//   E_bar = (1/N) sum E_mu,  o_k = (1/N) sum O_mu,k,  O~ = O - o   (centred in place)
//   S = (1/N) O~^T O~,       g = (1/N) O~^T (E - E_bar)
//   S_reg = S + diag(eps_rel S_kk + eps_abs); parameters with S_kk < freeze
//   are frozen (row/column of S_reg replaced by the identity, g_k = 0)
//   Delta alpha = -dtau S_reg^-1 g   by blocked Cholesky or by CG with the
//   matrix-free product S_reg v = (1/N) O~^T (O~ v) + shift v.
//
// All reductions run in a fixed order (row chunks summed by a second pass),
// so results are bitwise reproducible.  Every kernel is batched over
// instances (the last grid dimension) so ragged batches share launches.
#include <float.h>

#include <type_traits>

#include "sr.h"
#include "wave.h"

namespace mvmc {

// ------------------------------------------------------------ statistics
__global__ void k_estats(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.x];
  __shared__ double red[16];
  const double* e = A.eloc + I.eloc_off;
  const int64_t N = I.rows;
  double s = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += blockDim.x) s += e[m];
  s = block_sum(s, red);
  const double mean = s / (double)N;
  double v = 0.0;
  for (int64_t m = threadIdx.x; m < N; m += blockDim.x) {
    const double d = e[m] - mean;
    v += d * d;
  }
  v = block_sum(v, red);
  // standard error from the spread of the walker means (independent chains):
  // sigma = sqrt(sum_w (m_w - E_bar)^2 / (W (W - 1)))
  const int64_t W = I.walkers, ns = N / W;
  double d2 = 0.0;
  for (int64_t w = threadIdx.x; w < W; w += blockDim.x) {
    double mw = 0.0;
    for (int64_t s = 0; s < ns; ++s) mw += e[s * W + w];
    const double d = mw / (double)ns - mean;
    d2 += d * d;
  }
  d2 = block_sum(d2, red);
  if (threadIdx.x == 0) {
    A.scal[blockIdx.x * kScal + kEbar] = mean;
    A.scal[blockIdx.x * kScal + kEvar] = v / (double)N;
    A.scal[blockIdx.x * kScal + kEerr] = W > 1 ? sqrt(d2 / ((double)W * (double)(W - 1))) : NAN;
  }
}

// mode 0: partial column sums of O.  mode 1: centre O in place and form
// partial sums of O~^2 and O~ (E - E_bar); optionally write the bf16 split.
template <typename T>
__global__ void k_colpass(SrArgs A, T* __restrict__ O, int mode, uint16_t* __restrict__ split) {
  const SrInst& I = A.inst[blockIdx.z];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * kRowChunk;
  if (r0 >= I.rows) return;
  const int64_t r1 = r0 + kRowChunk < I.rows ? r0 + kRowChunk : I.rows;
  // rows up to the next multiple of 32 samples are read by the S kernels
  const int64_t rows32 = (I.rows + 31) / 32 * 32;
  const int64_t sld = I.split_ld;
  uint16_t* hi = (mode == 1 && split) ? split + I.split_off : nullptr;
  uint16_t* lo = hi ? hi + I.split_rows * sld : nullptr;
  if (k >= I.ldO) {
    // padding parameters of the split arrays (read by whole-tile loads): zero
    if (hi && k < sld) {
      const int64_t re = r1 == I.rows ? rows32 : r1;
      for (int64_t m = r0; m < re; ++m) {
        const int64_t si = split_index(m, k, sld);
        hi[si] = 0;
        lo[si] = 0;
      }
    }
    return;
  }
  T* Ob = O + I.O_off;
  double* part = A.colpart + I.colpart_off;
  const int64_t ld = I.ldO;
  if (mode == 0) {
    double s = 0.0;
    for (int64_t m = r0; m < r1; ++m) s += (double)Ob[m * ld + k];
    part[(blockIdx.y * 3 + 0) * ld + k] = s;
  } else {
    // padding columns (k >= np) hold zeros and have no mean of their own
    const double ob = k < I.np ? A.obar[I.param_off + k] : 0.0;
    const double eb = A.scal[blockIdx.z * kScal + kEbar];
    const double* e = A.eloc + I.eloc_off;
    double s2 = 0.0, sg = 0.0;
    for (int64_t m = r0; m < r1; ++m) {
      const T c = (T)((double)Ob[m * ld + k] - ob);
      Ob[m * ld + k] = c;
      const double cd = (double)c;
      s2 += cd * cd;
      sg += cd * (e[m] - eb);
      if (hi) {
        const uint16_t h = f32_to_bf16((float)c);
        const int64_t si = split_index(m, k, sld);
        hi[si] = h;
        lo[si] = f32_to_bf16((float)c - bf16_to_f32(h));
      }
    }
    if (hi && r1 == I.rows)
      for (int64_t m = I.rows; m < rows32; ++m) {
        const int64_t si = split_index(m, k, sld);
        hi[si] = 0;
        lo[si] = 0;
      }
    part[(blockIdx.y * 3 + 1) * ld + k] = s2;
    part[(blockIdx.y * 3 + 2) * ld + k] = sg;
  }
}

// Fixed-order sum of the row-chunk partials.
__global__ void k_colfinish(SrArgs A, int mode, double* __restrict__ g) {
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.ldO) return;
  const double* part = A.colpart + I.colpart_off;
  const int64_t ld = I.ldO;
  const int nch = (int)ceil_div<int64_t>(I.rows, kRowChunk);
  const double invN = 1.0 / (double)I.rows;
  if (mode == 0) {
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(c * 3 + 0) * ld + k];
    if (k < I.np) A.obar[I.param_off + k] = s * invN;
  } else {
    double s2 = 0.0, sg = 0.0;
    for (int c = 0; c < nch; ++c) {
      s2 += part[(c * 3 + 1) * ld + k];
      sg += part[(c * 3 + 2) * ld + k];
    }
    if (k < I.np) {
      A.sdiag[I.param_off + k] = s2 * invN;
      g[I.param_off + k] = sg * invN;
    }
  }
}

// ------------------------------------------------------ FP64 SYRK (vector)
// 64x64 upper-triangle tiles of S = O~^T O~ / N, split over row chunks.
constexpr int kTile = 64, kKc = 32;

__device__ __forceinline__ void tile_of(int t, int nt, int& ti, int& tj) {
  int row = 0, start = 0;
  while (t >= start + (nt - row)) {
    start += nt - row;
    ++row;
  }
  ti = row;
  tj = row + (t - start);
}

template <typename T>
__global__ __launch_bounds__(256) void k_syrk_vec(SrArgs A, const T* __restrict__ O) {
  const SrInst& I = A.inst[blockIdx.z];
  const int nt = (int)ceil_div<int64_t>(I.np, kTile);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= I.ksplit) return;
  int ti, tj;
  tile_of(blockIdx.x, nt, ti, tj);
  const int64_t chunk = ceil_div<int64_t>(ceil_div<int64_t>(I.rows, I.ksplit), kKc) * kKc;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < I.rows ? r0 + chunk : I.rows;
  __shared__ double As[kKc][kTile + 1];
  __shared__ double Bs[kKc][kTile + 1];
  const T* Ob = O + I.O_off;
  const int64_t ld = I.ldO;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  const int c_a = ti * kTile, c_b = tj * kTile;
  for (int64_t m0 = r0; m0 < r1; m0 += kKc) {
    for (int e = threadIdx.x; e < kKc * kTile; e += 256) {
      const int kk = e / kTile, c = e % kTile;
      const int64_t m = m0 + kk;
      const bool okm = m < r1;
      As[kk][c] = (okm && c_a + c < I.np) ? (double)Ob[m * ld + c_a + c] : 0.0;
      Bs[kk][c] = (okm && c_b + c < I.np) ? (double)Ob[m * ld + c_b + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kKc; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  double* part = A.syrkpart + I.syrkpart_off + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * kTile * kTile;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) part[(ty * 4 + i) * kTile + tx * 4 + j] = acc[i][j];
}

// Sum the split-K partials in order, scale by 1/N, write both triangles.
// Double-precision S on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// the same 64 x 64 upper-triangle tiles and sample split as k_syrk_vec, each
// wavefront a 32 x 32 quadrant as 2 x 2 blocks of 16 x 16 accumulators,
// operands read from the k-major LDS stage (16 consecutive doubles of one
// sample per MFMA operand).
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int kTp = kTile + 2;   // padded LDS row
__global__ __launch_bounds__(256) void k_syrk_f64mfma(SrArgs A, const double* __restrict__ O) {
  const SrInst& I = A.inst[blockIdx.z];
  if (I.wide64) return;   // k_syrk_f64_wide
  const int nt = (int)ceil_div<int64_t>(I.np, kTile);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles || (int)blockIdx.y >= I.ksplit) return;
  int ti, tj;
  tile_of(blockIdx.x, nt, ti, tj);
  const int64_t chunk = ceil_div<int64_t>(ceil_div<int64_t>(I.rows, I.ksplit), kKc) * kKc;
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  const int64_t r1 = r0 + chunk < I.rows ? r0 + chunk : I.rows;
  __shared__ double As[kKc][kTp];
  __shared__ double Bs[kKc][kTp];
  const double* Ob = O + I.O_off;
  const int64_t ld = I.ldO;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int qi = wv >> 1, qj = wv & 1, ka = lane >> 4, ma = lane & 15;
  const int c_a = ti * kTile, c_b = tj * kTile;
  f64x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  for (int64_t m0 = r0; m0 < r1; m0 += kKc) {
    for (int e = tid; e < kKc * kTile; e += 256) {
      const int kk = e / kTile, c = e % kTile;
      const int64_t m = m0 + kk;
      const bool okm = m < r1;
      As[kk][c] = (okm && c_a + c < I.np) ? Ob[m * ld + c_a + c] : 0.0;
      Bs[kk][c] = (okm && c_b + c < I.np) ? Ob[m * ld + c_b + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKc; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = As[kk + ka][32 * qi + 16 * i + ma];
        b[i] = Bs[kk + ka][32 * qj + 16 * i + ma];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // element r of lane l holds D[l / 16 + 4 r][l % 16] of its 16 x 16 block
  double* part = A.syrkpart + I.syrkpart_off + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * kTile * kTile;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        part[(32 * qi + 16 * i + ka + 4 * r) * kTile + 32 * qj + 16 * j + ma] = acc[i][j][r];
}

// Wide parameter sets in double precision: 128 x 128 upper-triangle tiles
// straight into S (both triangles, scaled by 1/N), no sample split.  Four
// wavefronts, each a 64 x 64 quadrant as 4 x 4 blocks of 16 x 16 MFMA
// accumulators; the samples pass through LDS sixteen at a time as they lie in
// O (sample-major rows, so every MFMA operand is 16 consecutive parameters of
// one sample), double-buffered through registers.  O's padding columns are
// zero, so only samples past N need masking.  The lower triangle is written
// from each 16 x 16 block transposed through LDS, so both writes are
// coalesced.  The tiles past the last full round of workgroups (from nfull
// on) are split into tail_ks sample parts, whose unscaled partial tiles go to
// the partial pool and are summed in part order by k_syrk_f64_tail, so the
// last round is as full as the others.
constexpr int kWT = 128, kWK = 16, kWP = kWT + 2;
__global__ __launch_bounds__(256, 2) void k_syrk_f64_wide(SrArgs A, const double* __restrict__ O,
                                                          double* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.y];
  if (!I.wide64) return;
  const int nt = (int)ceil_div<int64_t>(I.np, kWT);
  const int ntl = nt * (nt + 1) / 2;
  const int u = (int)blockIdx.x;
  if (u >= I.nfull + (ntl - I.nfull) * I.tail_ks) return;
  // unit u: a whole tile (u < nfull) or sample part pk of tail tile t
  const int t = u < I.nfull ? u : I.nfull + (u - I.nfull) / I.tail_ks;
  const int pk = u < I.nfull ? -1 : (u - I.nfull) % I.tail_ks;
  int ti, tj;
  tile_of(t, nt, ti, tj);   // ti <= tj
  const int64_t ca = (int64_t)ti * kWT, cb = (int64_t)tj * kWT, ld = I.ldO, rows = I.rows;
  int64_t mb = 0, me = rows;   // samples of this unit (part bounds on kWK steps)
  double* part = nullptr;
  if (pk >= 0) {
    const int64_t steps = ceil_div<int64_t>(rows, kWK);
    const int64_t chunk = ceil_div<int64_t>(steps, I.tail_ks) * kWK;
    mb = pk * chunk;
    me = mb + chunk < rows ? mb + chunk : rows;
    part = A.syrkpart + I.syrkpart_off + ((int64_t)(t - I.nfull) * I.tail_ks + pk) * kWT * kWT;
    if (mb >= me) {   // empty part: contributes zero
      for (int e = threadIdx.x; e < kWT * kWT; e += blockDim.x) part[e] = 0.0;
      return;
    }
  }
  const double* Ob = O + I.O_off;
  __shared__ double As[2][kWK][kWP];
  __shared__ double Bs[2][kWK][kWP];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int qi = wv >> 1, qj = wv & 1;
  const int lk = tid >> 4, lc = (tid & 15) * 8;   // staging: sample lk, parameters lc..lc+7
  double ga[8], gb[8];
  auto gload = [&](int64_t m0) {
    const int64_t m = m0 + lk;
    const bool ok = m < rows;
    const double* pa = Ob + (ok ? m : 0) * ld + ca + lc;
    const double* pb = Ob + (ok ? m : 0) * ld + cb + lc;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ga[e] = ok ? pa[e] : 0.0;
      gb[e] = ok ? pb[e] : 0.0;
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[st][lk][lc + e] = ga[e];
      Bs[st][lk][lc + e] = gb[e];
    }
  };
  f64x4_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  gload(mb);
  lstore(0);
  __syncthreads();
  int st = 0;
  const int ka = lane >> 4, ma = lane & 15;
  for (int64_t m0 = mb; m0 < me; m0 += kWK) {
    const bool more = m0 + kWK < me;
    if (more) gload(m0 + kWK);
#pragma unroll
    for (int kk = 0; kk < kWK; kk += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[st][kk + ka][64 * qi + 16 * i + ma];
        b[i] = Bs[st][kk + ka][64 * qj + 16 * i + ma];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) lstore(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
  // element r of lane l holds D[l / 16 + 4 r][l % 16] of its 16 x 16 block
  if (part) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          part[(64 * qi + 16 * i + ka + 4 * r) * kWT + 64 * qj + 16 * j + ma] = acc[i][j][r];
    return;
  }
  const double invN = 1.0 / (double)rows;
  double* Sb = S + I.S_off;
  const int64_t np = I.np;
  double* tr = &As[0][0][0] + wv * 16 * 17;   // per-wavefront 16 x 17 transpose buffer
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t rb = ca + 64 * qi + 16 * i, cbb = cb + 64 * qj + 16 * j;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rb + ka + 4 * r, col = cbb + ma;
        const double v = acc[i][j][r] * invN;
        if (row < np && col < np) Sb[row * np + col] = v;
        tr[(ka + 4 * r) * 17 + ma] = v;
      }
      if (ti != tj) {   // mirror: row col of S gets this block's column
        wave::wave_sync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = cbb + ka + 4 * r, col = rb + ma;   // S[row][col] = D[col - rb][row - cbb]
          const double v = tr[ma * 17 + ka + 4 * r];
          if (row < np && col < np) Sb[row * np + col] = v;
        }
        wave::wave_sync();
      }
    }
}

// Tail tiles of k_syrk_f64_wide: the sample parts summed in order, scaled by
// 1/N, written to both triangles (a diagonal tile holds both already).
__global__ __launch_bounds__(256) void k_syrk_f64_tail(SrArgs A, double* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.z];
  if (!I.wide64 || I.tail_ks < 2) return;
  const int nt = (int)ceil_div<int64_t>(I.np, kWT);
  const int tt = I.nfull + (int)blockIdx.y;
  if (tt >= nt * (nt + 1) / 2) return;
  const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;   // grid covers kWT^2 exactly
  int ti, tj;
  tile_of(tt, nt, ti, tj);
  const int64_t row = (int64_t)ti * kWT + e / kWT, col = (int64_t)tj * kWT + e % kWT;
  if (row >= I.np || col >= I.np) return;
  const double* part = A.syrkpart + I.syrkpart_off + (int64_t)blockIdx.y * I.tail_ks * kWT * kWT;
  double a = 0.0;
  for (int k = 0; k < I.tail_ks; ++k) a += part[(int64_t)k * kWT * kWT + e];
  const double v = a * (1.0 / (double)I.rows);
  double* Sb = S + I.S_off;
  Sb[row * I.np + col] = v;
  if (ti != tj) Sb[col * I.np + row] = v;
}

template <typename TS>
__global__ void k_syrk_reduce(SrArgs A, TS* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.z];
  if (I.wide64) return;
  const int nt = (int)ceil_div<int64_t>(I.np, kTile);
  const int ntiles = nt * (nt + 1) / 2;
  if ((int)blockIdx.x >= ntiles) return;
  int ti, tj;
  tile_of(blockIdx.x, nt, ti, tj);
  const double* part = A.syrkpart + I.syrkpart_off;
  const double invN = 1.0 / (double)I.rows;
  TS* Sb = S + I.S_off;
  const int e = (int)blockIdx.y * blockDim.x + threadIdx.x;   // element of the tile
  if (e >= kTile * kTile) return;
  const int i = e / kTile, j = e % kTile;
  const int64_t r = (int64_t)ti * kTile + i, c = (int64_t)tj * kTile + j;
  if (r >= I.np || c >= I.np) return;
  double s = 0.0;
  for (int ks = 0; ks < I.ksplit; ++ks) s += part[((int64_t)ks * ntiles + blockIdx.x) * kTile * kTile + e];
  s *= invN;
  Sb[r * I.np + c] = (TS)s;
  Sb[c * I.np + r] = (TS)s;
}

// ------------------------------------------------------------ SR solve
// Regularised matrix into the FP64 factor pool (lower triangle and diagonal)
// and the masked right-hand side into x.
template <typename TS>
__global__ void k_chol_prep(SrArgs A, const TS* __restrict__ S, const double* __restrict__ g,
                            double eps_rel, double eps_abs, double freeze) {
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t r = blockIdx.x;
  if (r >= I.np) return;
  const double* d = A.sdiag + I.param_off;
  const bool kr = d[r] >= freeze;
  double* F = A.chol + I.chol_off + r * I.np;
  const TS* Sr = S + I.S_off + r * I.np;
  for (int64_t c = threadIdx.x; c <= r; c += blockDim.x) {
    const bool kc = d[c] >= freeze;
    double v = (kr && kc) ? (double)Sr[c] : 0.0;
    if (c == r) v += kr ? eps_rel * d[r] + eps_abs : 1.0;
    F[c] = v;
  }
  if (threadIdx.x == 0) A.x[I.param_off + r] = kr ? g[I.param_off + r] : 0.0;
}

constexpr int kNb = 64;

namespace {
__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
}  // namespace

// One block column of the factor and of the forward substitution per
// launch.  Within an outer panel the factor is left-looking: block column kb
// still lacks the contributions of the panel's earlier columns c (kb0 <= c <
// kb); the columns of earlier panels were applied by k_chol_trail.  Workgroup
// b of an instance owns row block ib = kb + b and computes
//   D = F[kb][kb] - sum_c L[kb][c] L[kb][c]^T        (every workgroup; 64 x 64)
//   L_kk = chol(D),  y_kb = L_kk^-1 x_kb              (forward substitution)
// and then, for ib == kb, stores L_kk and y_kb (into r), or for ib > kb
//   B = F[ib][kb] - sum_c L[ib][c] L[kb][c]^T,   L[ib][kb] = B L_kk^-T,
//   x_ib -= L[ib][kb] y_kb.
// The sums over c run on the FP64 matrix cores.  The 64 x 64 factor runs
// in four steps over column strips of 16: the
// strip's 16 x 16 diagonal block by Crout in 16 lanes,
//   L[i][j] = (D[i][j] - sum_{m<j} L[i][m] L[j][m]) / L[j][j],
//   L[j][j] = sqrt(D[j][j] - sum_{m<j} L[j][m]^2),
// then every row below it in the strip, every row of B and the row x_kb^T
// by the same 16-step recurrence against that block (one thread per row),
// then the update of the columns right of the strip; B's rows end as
// B L_kk^-T and the last row as y_kb^T.  Blocks past the matrix are padded
// with the identity.  L_kk is stored in block kb's slot after the factor
// (chol_off + np^2 + kb 64^2, row-major), never in F: the other workgroups of
// the launch still read F[kb][kb].  A non-positive pivot sets the instance's
// flag.
constexpr int kColPad = kNb + 1;   // row stride of the factor phase (2-way LDS banks)
constexpr int kGemmPad = kNb + 2;  // row stride of the k-major stage (16-byte aligned rows)
constexpr int kStrip = 16;
typedef double f64x2 __attribute__((ext_vector_type(2)));

// 1/sqrt(d) for d > 0 to double precision: the hardware estimate and two
// Newton steps y <- y (3 - d y^2) / 2 (each doubles the correct bits).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * (1.5 - 0.5 * d * y * y);
  y = y * (1.5 - 0.5 * d * y * y);
  return y;
}

__global__ __launch_bounds__(256) void k_chol_column(SrArgs A, int kb, int kb0) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  if (kb >= nblk) return;
  const int ib = kb + (int)blockIdx.x;
  if (ib >= nblk) return;
  const bool diag = ib == kb;
  const int64_t o = (int64_t)kb * kNb, ro = (int64_t)ib * kNb, np = I.np;
  const int nb = (int)(np - o < kNb ? np - o : kNb);
  const int nr = (int)(np - ro < kNb ? np - ro : kNb);
  double* F = A.chol + I.chol_off;
  double* x = A.x + I.param_off;
  // two LDS regions, each viewed k-major for the GEMM stage and row-major
  // for the factor phase
  __shared__ __align__(16) double bufP[kNb * kGemmPad];         // L[kb][c]^T, then D and L_kk
  __shared__ __align__(16) double bufQ[(kNb + 1) * kGemmPad];   // L[ib][c]^T, then B and x_kb^T
  __shared__ double rd[kNb];                                    // 1 / L_kk[j][j]
  auto P = reinterpret_cast<double (*)[kColPad]>(bufP);
  auto Q = reinterpret_cast<double (*)[kColPad]>(bufQ);
  auto Pt = reinterpret_cast<double (*)[kGemmPad]>(bufP);
  auto Qt = reinterpret_cast<double (*)[kGemmPad]>(bufQ);
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  // in-panel update on the FP64 matrix cores: wavefront wv owns the 32 x 32
  // quadrant (qi, qj) of D and B, 2 x 2 blocks of 16 x 16 (element r of lane
  // l is row l / 16 + 4 r, column l % 16 of its block); an operand is 16
  // consecutive doubles of one k row of the staged chunk
  const int qi = wv >> 1, qj = wv & 1, ka = lane >> 4, ma = lane & 15;
  f64x4_t accD[2][2], accB[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accD[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
      accB[i][j] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    }
  // D is needed on and below its diagonal: the quadrant above it is skipped
  const bool needD = qi >= qj;
  // 64 x 64 x 64 products per earlier column block (full blocks), operands
  // staged k-major
  for (int c = kb0; c < kb; ++c) {
    const int64_t co = (int64_t)c * kNb;
    // every load of the chunk in flight before the first LDS store
    constexpr int kU = kNb * kNb / 256;
    double vp[kU], vq[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = tid + 256 * u, i = e / kNb, k = e % kNb;
      vp[u] = i < nb ? F[(o + i) * np + co + k] : 0.0;
      vq[u] = (!diag && i < nr) ? F[(ro + i) * np + co + k] : 0.0;
    }
    __syncthreads();   // the previous chunk is consumed
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = tid + 256 * u, i = e / kNb, k = e % kNb;
      Pt[k][i] = vp[u];
      Qt[k][i] = vq[u];
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kNb; kk += 4) {
      double pa[2], pb[2], qa[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        pa[i] = Pt[kk + ka][32 * qi + 16 * i + ma];
        pb[i] = Pt[kk + ka][32 * qj + 16 * i + ma];
        qa[i] = Qt[kk + ka][32 * qi + 16 * i + ma];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (needD) accD[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[i], pb[j], accD[i][j], 0, 0, 0);
          if (!diag) accB[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[i], pb[j], accB[i][j], 0, 0, 0);
        }
    }
  }
  // D (lower triangle, identity past the matrix), B and x_kb^T; the loads
  // first, all in flight
  double fd[2][2][4], fb[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 32 * qi + 16 * i + ka + 4 * q, cc = 32 * qj + 16 * j + ma;
        fd[i][j][q] = (r < nb && cc <= r) ? F[(o + r) * np + o + cc] : 0.0;
        fb[i][j][q] = (!diag && r < nr && cc < nb) ? F[(ro + r) * np + o + cc] : 0.0;
      }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 32 * qi + 16 * i + ka + 4 * q, cc = 32 * qj + 16 * j + ma;
        double d;
        if (r < nb && cc < nb) d = cc <= r ? fd[i][j][q] - accD[i][j][q] : 0.0;
        else d = r == cc ? 1.0 : 0.0;
        P[r][cc] = d;
        if (!diag) Q[r][cc] = (r < nr && cc < nb) ? fb[i][j][q] - accB[i][j][q] : 0.0;
      }
  if (tid < kNb) Q[kNb][tid] = tid < nb ? x[o + tid] : 0.0;
  const int q0 = diag ? kNb : 0;   // first row of Q to solve (the diagonal block solves x only)
  bool bad = false;
  for (int c0 = 0; c0 < kNb; c0 += kStrip) {
    __syncthreads();
    if (tid < kStrip) {   // the strip's diagonal block, lanes 0..15 of wavefront 0
      const int i = tid;
      double rr[kStrip];
#pragma unroll
      for (int j = 0; j < kStrip; ++j) rr[j] = P[c0 + i][c0 + j];
#pragma unroll
      for (int j = 0; j < kStrip; ++j) {
        double s0 = rr[j], s1 = 0.0;
#pragma unroll
        for (int m = 0; m < j; ++m) {
          if (m & 1) s1 -= rr[m] * P[c0 + j][c0 + m];
          else s0 -= rr[m] * P[c0 + j][c0 + m];
        }
        const double sv = s0 + s1;
        const double dj = lane_value(sv, j);
        if (c0 + j < nb && !(dj > 0.0)) bad = true;
        const double rl = rsqrt_nr(dj > 0.0 ? dj : DBL_MIN);   // 1 / L[j][j]
        rr[j] = i == j ? (dj > 0.0 ? dj : DBL_MIN) * rl : sv * rl;
        if (j <= i) P[c0 + i][c0 + j] = rr[j];
        if (i == j) rd[c0 + j] = rl;
        wave::wave_sync();
        asm volatile("" ::: "memory");   // row j is complete before step j + 1 reads it
      }
    }
    __syncthreads();
    // rows below the block in the strip, then the rows of Q, one thread each
    const int nbelow = kNb - c0 - kStrip;
    const int nrows = nbelow + (kNb + 1 - q0);
    if (tid < nrows) {
      double* row = tid < nbelow ? &P[c0 + kStrip + tid][0] : &Q[q0 + tid - nbelow][0];
      double t[kStrip];
#pragma unroll
      for (int j = 0; j < kStrip; ++j) t[j] = row[c0 + j];
#pragma unroll
      for (int j = 0; j < kStrip; ++j) {
        double s0 = t[j], s1 = 0.0;
#pragma unroll
        for (int m = 0; m < j; ++m) {
          if (m & 1) s1 -= t[m] * P[c0 + j][c0 + m];
          else s0 -= t[m] * P[c0 + j][c0 + m];
        }
        t[j] = (s0 + s1) * rd[c0 + j];
      }
#pragma unroll
      for (int j = 0; j < kStrip; ++j) row[c0 + j] = t[j];
    }
    __syncthreads();
    // columns right of the strip, 2 x 2 entries per task: P[r][cc] (cc <= r)
    // and Q[r][cc]
    const int c1 = c0 + kStrip;
    const int hb = nbelow / 2;                          // column pairs
    const int qrows = kNb + 1 - q0;
    const int nP = hb * hb, nQ = ((qrows + 1) / 2) * hb;
    for (int e = tid; e < nP + nQ; e += 256) {
      const double* r0p;
      const double* r1p;
      double* w0;
      double* w1;
      int cc;
      bool tri = false;
      if (e < nP) {
        const int rp = e / hb, cp = e % hb;
        if (cp > rp) continue;
        const int r = c1 + 2 * rp;
        cc = c1 + 2 * cp;
        w0 = &P[r][0];
        w1 = &P[r + 1][0];
        tri = cp == rp;   // the 2 x 2 block on the diagonal: skip its upper entry
      } else {
        const int u = e - nP, rp = u / hb;
        cc = c1 + 2 * (u % hb);
        const int r = q0 + 2 * rp;
        w0 = &Q[r][0];
        w1 = r + 1 < kNb + 1 ? &Q[r + 1][0] : nullptr;
      }
      r0p = w0;
      r1p = w1 ? w1 : w0;
      double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
#pragma unroll
      for (int m = 0; m < kStrip; ++m) {
        const double x0 = r0p[c0 + m], x1 = r1p[c0 + m];
        const double y0 = P[cc][c0 + m], y1 = P[cc + 1][c0 + m];
        s00 += x0 * y0;
        s01 += x0 * y1;
        s10 += x1 * y0;
        s11 += x1 * y1;
      }
      w0[cc] -= s00;
      if (!tri) w0[cc + 1] -= s01;
      if (w1) {
        w1[cc] -= s10;
        w1[cc + 1] -= s11;
      }
    }
  }
  if (bad && diag) A.scal[blockIdx.y * kScal + kFlag] = 1.0;
  __syncthreads();
  if (diag) {
    double* Lk = F + np * np + (int64_t)kb * kNb * kNb;
    for (int e = tid; e < kNb * kNb; e += 256) {
      const int i = e / kNb, j = e % kNb;
      Lk[e] = j <= i ? P[i][j] : 0.0;
    }
    if (tid < nb) A.r[I.param_off + o + tid] = Q[kNb][tid];
  } else {
    for (int e = tid; e < kNb * kNb; e += 256) {
      const int i = e / kNb, j = e % kNb;
      if (i < nr && j < nb) F[(ro + i) * np + o + j] = Q[i][j];
    }
    if (tid < nr) {
      double cacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int j = 0; j < kNb; ++j) cacc[j & 3] += Q[tid][j] * Q[kNb][j];
      x[ro + tid] -= (cacc[0] + cacc[1]) + (cacc[2] + cacc[3]);
    }
  }
}

// Trailing update of outer step ob: the lower triangle of the rows and
// columns past the outer panel [o, o + kOuter) less L[:, panel] L[:, panel]^T,
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64), accumulated onto the
// tile's values loaded at the start.  A workgroup of four
// wavefronts owns a UT x UT tile, each wavefront a UT/2 x UT/2 quadrant of
// 16 x 16 accumulator blocks.  The panel's columns pass through
// LDS k-major (each MFMA operand is 16 consecutive doubles of one column),
// 16 at a time, double-buffered; rows past the matrix read the last row.
// Two workgroups share a compute unit (two wavefronts per SIMD), which the
// FP64 matrix unit needs to stay busy.
constexpr int kOuter = 4 * kNb;   // outer panel width
constexpr int kUK = 16;           // panel columns per LDS stage
typedef double f64x4 __attribute__((ext_vector_type(4)));

// UT: tile side, 128 (each wavefront 4 x 4 blocks) or 64 (2 x 2 blocks, for
// the small trailing matrices of the last panels, where 128-tiles leave most
// compute units idle).
template <int UT>
__global__ __launch_bounds__(256, 2) void k_chol_trail(SrArgs A, int ob) {
  constexpr int UP = UT + 2;            // padded LDS row (spreads the four k rows of an operand over the banks)
  constexpr int QB = UT / 32;           // 16 x 16 blocks per side of a wavefront's quadrant
  constexpr int EL = kUK * UT / 256;    // staged values per thread and stage
  constexpr int TPR = kUK / EL;         // threads per staged row
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t o = (int64_t)ob * kOuter, t0 = o + kOuter;
  if (t0 >= I.np) return;
  const int nt = (int)ceil_div<int64_t>(I.np - t0, UT);
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int ti = 0, start = 0;   // lower-triangle tile (ti >= tj)
  while ((int)blockIdx.x >= start + ti + 1) {
    start += ti + 1;
    ++ti;
  }
  const int tj = (int)blockIdx.x - start;
  const int64_t r0 = t0 + (int64_t)ti * UT, c0 = t0 + (int64_t)tj * UT;
  double* F = A.chol + I.chol_off;
  __shared__ double As[2][kUK][UP];
  __shared__ double Bs[2][kUK][UP];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int qi = wv >> 1, qj = wv & 1;
  const int lr = tid / TPR, lk = (tid % TPR) * EL;   // staging: EL values of row lr
  const int64_t ra = r0 + lr, rb = c0 + lr;
  const double* pa = F + (ra < I.np ? ra : I.np - 1) * I.np + o + lk;
  const double* pb = F + (rb < I.np ? rb : I.np - 1) * I.np + o + lk;
  double ga[EL], gb[EL];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      ga[e] = pa[k0 + e];
      gb[e] = pb[k0 + e];
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      As[st][lk + e][lr] = ga[e];
      Bs[st][lk + e][lr] = gb[e];
    }
  };
  const int ka = lane >> 4, ma = lane & 15;   // operand element: k row, row within the block
  // the accumulators start from the tile's current values (element r of lane
  // l is D[l / 16 + 4 r][l % 16] of its 16 x 16 block) and take the panel's
  // products with one operand negated, so the tile is written once at the
  // end and never read there
  f64x4 acc[QB][QB];
#pragma unroll
  for (int i = 0; i < QB; ++i)
#pragma unroll
    for (int j = 0; j < QB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + (UT / 2) * qi + 16 * i + ka + 4 * r;
        const int64_t col = c0 + (UT / 2) * qj + 16 * j + ma;
        acc[i][j][r] = (row < I.np && col < I.np) ? F[row * I.np + col] : 0.0;
      }
  gload(0);
  lstore(0);
  __syncthreads();
  int st = 0;
  for (int k0 = 0; k0 < kOuter; k0 += kUK) {
    const bool more = k0 + kUK < kOuter;
    if (more) gload(k0 + kUK);
#pragma unroll
    for (int kk = 0; kk < kUK; kk += 4) {
      double a[QB], b[QB];
#pragma unroll
      for (int i = 0; i < QB; ++i) {
        a[i] = -As[st][kk + ka][(UT / 2) * qi + 16 * i + ma];
        b[i] = Bs[st][kk + ka][(UT / 2) * qj + 16 * i + ma];
      }
#pragma unroll
      for (int i = 0; i < QB; ++i)
#pragma unroll
        for (int j = 0; j < QB; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) lstore(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
#pragma unroll
  for (int i = 0; i < QB; ++i)
#pragma unroll
    for (int j = 0; j < QB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + (UT / 2) * qi + 16 * i + ka + 4 * r;
        const int64_t col = c0 + (UT / 2) * qj + 16 * j + ma;
        if (row < I.np && col < I.np && (ti != tj || col <= row)) F[row * I.np + col] = acc[i][j][r];
      }
}

// Inverse of every 64 x 64 diagonal block of the factor, all blocks at once
// (one wavefront each), in place in the slots after the factor
// (chol_off + np^2 + kb * 64^2, row-major, where k_chol_column left L_kk).
// Lane j forms column j by forward substitution, L z = e_j:
// z_i = (delta_ij - sum_{m<i} L[i][m] z_m) / L[i][i], with L_kk and the
// columns in LDS.  Rows and columns past the matrix (last block) are the
// identity.
__global__ __launch_bounds__(64) void k_trtri_diag(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  const int kb = blockIdx.x;
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  if (kb >= nblk) return;
  const int64_t o = (int64_t)kb * kNb;
  const int nb = (int)(I.np - o < kNb ? I.np - o : kNb);
  double* Li = A.chol + I.chol_off + I.np * I.np + (int64_t)kb * kNb * kNb;
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double Zs[kNb][kNb + 1];
  const int j = threadIdx.x;
  for (int i = 0; i < kNb; ++i) {
    Ls[i][j] = (i < nb && j <= i) ? Li[i * kNb + j] : (i == j ? 1.0 : 0.0);
    Zs[i][j] = 0.0;
  }
  wave::wave_sync();
  for (int i = 0; i < kNb; ++i) {
    double s = i == j ? 1.0 : 0.0;
    for (int m = j; m < i; ++m) s -= Ls[i][m] * Zs[m][j];
    Zs[i][j] = i < j ? 0.0 : s / Ls[i][i];
  }
  wave::wave_sync();
  for (int i = 0; i < kNb; ++i) Li[i * kNb + j] = Zs[i][j];
}

// Backward substitution L^T x = y (y left in r by k_chol_column), one block
// row per launch from each instance's own last block: step s solves block
// b = nblk - 1 - s, whose y_b is final (every later block's contribution
// was applied by the earlier steps).  Every workgroup forms
//   x_b = Linv_bb^T y_b            (the inverted diagonal block, k_trtri_diag)
// workgroup 0 stores it, and workgroup t < b applies
//   y_t -= L[b][t]^T x_b.
// The four wavefronts split the 64 rows of each 64 x 64 block, lanes across
// its columns (coalesced), partial sums added in wavefront order.
__global__ __launch_bounds__(256) void k_trsv_back(SrArgs A, int step) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  const int b = nblk - 1 - step;
  const int t = (int)blockIdx.x;
  if (b < 0 || (t > 0 && t >= b)) return;
  const int64_t np = I.np, ob = (int64_t)b * kNb;
  const int nb = (int)(np - ob < kNb ? np - ob : kNb);
  const double* F = A.chol + I.chol_off;
  const double* Li = F + np * np + (int64_t)b * kNb * kNb;
  double* y = A.r + I.param_off;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int kR = kNb / 4;   // rows per wavefront
  __shared__ double part[4][kNb];
  __shared__ double xb[kNb];
  double li[kR], yb[kR];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    const int i = wv * kR + u;
    li[u] = Li[i * kNb + lane];
    yb[u] = i < nb ? y[ob + i] : 0.0;
  }
  double acc = 0.0;
#pragma unroll
  for (int u = 0; u < kR; ++u) acc += li[u] * yb[u];
  part[wv][lane] = acc;
  __syncthreads();
  if (tid < kNb) xb[tid] = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
  __syncthreads();
  if (t == 0 && tid < nb) A.x[I.param_off + ob + tid] = xb[tid];
  if (t >= b) return;   // uniform per workgroup
  const int64_t ot = (int64_t)t * kNb;   // a full block (t < b)
  double lv[kR];
#pragma unroll
  for (int u = 0; u < kR; ++u) {
    const int i = wv * kR + u;
    lv[u] = i < nb ? F[(ob + i) * np + ot + lane] : 0.0;
  }
  acc = 0.0;
#pragma unroll
  for (int u = 0; u < kR; ++u) acc += lv[u] * xb[wv * kR + u];
  __syncthreads();   // part is free
  part[wv][lane] = acc;
  __syncthreads();
  if (tid < kNb) y[ot + tid] -= ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
}

// ------------------------------------------------------------------- CG
// Algorithm 1 with A = S_reg applied matrix-free.
__global__ void k_cg_init(SrArgs A, const double* __restrict__ g, double eps_rel, double eps_abs,
                          double freeze) {
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.np) return;
  const int64_t o = I.param_off + k;
  const double d = A.sdiag[o];
  const bool keep = d >= freeze;
  const double b = keep ? g[o] : 0.0;
  A.x[o] = 0.0;
  A.r[o] = b;
  A.p[o] = b;
  A.shift[o] = keep ? eps_rel * d + eps_abs : 1.0;
  A.mask[o] = keep ? 1.0 : 0.0;
}

// out = a . b per instance in two fixed-order passes: chunk partial sums
// over up to kDotParts workgroups (chunks of at least 4096 entries), then
// their sum in chunk order.
__device__ __forceinline__ int dot_parts(int64_t np) {
  const int64_t p = ceil_div<int64_t>(np, 4096);
  return (int)(p < kDotParts ? (p > 0 ? p : 1) : kDotParts);
}

__global__ __launch_bounds__(256) void k_dot_part(SrArgs A, const double* __restrict__ a,
                                                  const double* __restrict__ b, int check_done) {
  const SrInst& I = A.inst[blockIdx.y];
  if (check_done && A.scal[blockIdx.y * kScal + kDone] != 0.0) return;
  const int parts = dot_parts(I.np);
  if ((int)blockIdx.x >= parts) return;
  const int64_t chunk = ceil_div<int64_t>(I.np, parts);
  const int64_t k0 = (int64_t)blockIdx.x * chunk;
  const int64_t k1 = k0 + chunk < I.np ? k0 + chunk : I.np;
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t k = k0 + threadIdx.x; k < k1; k += blockDim.x)
    s += a[I.param_off + k] * b[I.param_off + k];
  s = block_sum(s, red);
  if (threadIdx.x == 0) A.dotpart[(int64_t)blockIdx.y * kDotParts + blockIdx.x] = s;
}

__global__ void k_dot_finish(SrArgs A, int slot, int check_done) {
  const SrInst& I = A.inst[blockIdx.x];
  if (check_done && A.scal[blockIdx.x * kScal + kDone] != 0.0) return;
  if (threadIdx.x != 0) return;
  const double* pp = A.dotpart + (int64_t)blockIdx.x * kDotParts;
  const int parts = dot_parts(I.np);
  double s = 0.0;
  for (int q = 0; q < parts; ++q) s += pp[q];
  A.scal[blockIdx.x * kScal + slot] = s;
}

// t = O~ (mask o p).  A wavefront takes kRowsPerWave sample rows (one read
// of mask o p serves them all) over one chunk of kColChunk parameters; wide
// rows are split into chunks whose partial sums go to the upper third of the
// column-statistics buffer and are added in chunk order by k_gemv_rows_finish.
constexpr int kRowsPerWave = 4;
constexpr int kColChunk = 4096;
__device__ __forceinline__ int64_t row_chunks(int64_t np) { return ceil_div<int64_t>(np, kColChunk); }

template <typename T>
__global__ __launch_bounds__(256) void k_gemv_rows(SrArgs A, const T* __restrict__ O) {
  const SrInst& I = A.inst[blockIdx.z];
  if (A.scal[blockIdx.z * kScal + kDone] != 0.0) return;
  const int64_t nch = row_chunks(I.np);
  if ((int64_t)blockIdx.y >= nch) return;
  const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kRowsPerWave;
  if (m0 >= I.rows) return;
  const int lane = threadIdx.x & 63;
  const int64_t c0 = (int64_t)blockIdx.y * kColChunk;
  const int64_t c1 = c0 + kColChunk < I.np ? c0 + kColChunk : I.np;
  const T* row = O + I.O_off + m0 * I.ldO;
  const double* p = A.p + I.param_off;
  const double* mk = A.mask + I.param_off;
  const int nr = I.rows - m0 < kRowsPerWave ? (int)(I.rows - m0) : kRowsPerWave;
  double s[kRowsPerWave] = {};
  if constexpr (sizeof(T) == 4) {
    // single precision: four consecutive elements per lane and 16-byte
    // load (the row stride and offsets are multiples of 64 elements), the
    // ragged end of the chunk one element at a time
    typedef float vec_t __attribute__((ext_vector_type(4)));
#pragma unroll 2
    for (int64_t k0 = c0 + 4 * lane; k0 < c1; k0 += 256) {
      if (k0 + 4 <= c1) {
        double pk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) pk[j] = p[k0 + j] * mk[k0 + j];
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r)
          if (r < nr) {
            const vec_t v = *reinterpret_cast<const vec_t*>(row + r * I.ldO + k0);
#pragma unroll
            for (int j = 0; j < 4; ++j) s[r] += (double)v[j] * pk[j];
          }
      } else {
        for (int64_t k = k0; k < c1; ++k) {
          const double pk = p[k] * mk[k];
#pragma unroll
          for (int r = 0; r < kRowsPerWave; ++r)
            if (r < nr) s[r] += (double)row[r * I.ldO + k] * pk;
        }
      }
    }
  } else {
    // double: one element per lane, 512 bytes per wave and load
#pragma unroll 4
    for (int64_t k = c0 + lane; k < c1; k += 64) {
      const double pk = p[k] * mk[k];
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r)
        if (r < nr) s[r] += (double)row[r * I.ldO + k] * pk;
    }
  }
  double* part = A.colpart + I.colpart_off +
                 2 * ceil_div<int64_t>(I.rows, kRowChunk) * I.ldO;   // upper third
#pragma unroll
  for (int r = 0; r < kRowsPerWave; ++r) {
    const double v = wave_sum(s[r]);
    if (lane == 0 && r < nr) {
      if (nch == 1) A.t[I.eloc_off + m0 + r] = v;
      else part[(int64_t)blockIdx.y * I.rows + m0 + r] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_gemv_rows_finish(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  if (A.scal[blockIdx.y * kScal + kDone] != 0.0) return;
  const int64_t nch = row_chunks(I.np);
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (nch == 1 || m >= I.rows) return;
  const double* part = A.colpart + I.colpart_off + 2 * ceil_div<int64_t>(I.rows, kRowChunk) * I.ldO;
  double s = 0.0;
  for (int64_t c = 0; c < nch; ++c) s += part[c * I.rows + m];
  A.t[I.eloc_off + m] = s;
}

// w = mask o (O~^T t) / N + shift o p, in two passes: partial sums over
// chunks of kRowChunk rows (a workgroup covers 64 columns, its four waves
// interleave the rows of the chunk, coalesced along the columns), then the
// chunk partials summed in chunk order.  The partial buffer of the column
// statistics is free once they have been reduced.
template <typename T>
__global__ __launch_bounds__(256) void k_gemv_cols_part(SrArgs A, const T* __restrict__ O) {
  // each lane takes 16 bytes of columns (the row stride and offsets are
  // multiples of 64 elements); the four wavefronts split the rows
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(VW)));
  const SrInst& I = A.inst[blockIdx.z];
  if (A.scal[blockIdx.z * kScal + kDone] != 0.0) return;
  const int64_t m0 = (int64_t)blockIdx.y * kRowChunk;
  if (m0 >= I.rows) return;
  const int64_t m1 = m0 + kRowChunk < I.rows ? m0 + kRowChunk : I.rows;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t k0 = ((int64_t)blockIdx.x * 64 + lane) * VW;
  const double* t = A.t + I.eloc_off;
  double s[VW] = {};
  if (k0 < I.np) {
    const T* col = O + I.O_off + k0;
#pragma unroll 4
    for (int64_t m = m0 + wv; m < m1; m += 4) {
      const vec_t v = *reinterpret_cast<const vec_t*>(col + m * I.ldO);
      const double tm = t[m];
#pragma unroll
      for (int j = 0; j < VW; ++j) s[j] += (double)v[j] * tm;
    }
  }
  __shared__ double red[4][VW][64];
#pragma unroll
  for (int j = 0; j < VW; ++j) red[wv][j][lane] = s[j];
  __syncthreads();
  if (wv == 0)
#pragma unroll
    for (int j = 0; j < VW; ++j)
      if (k0 + j < I.np)
        A.colpart[I.colpart_off + (int64_t)blockIdx.y * I.np + k0 + j] =
            (red[0][j][lane] + red[1][j][lane]) + (red[2][j][lane] + red[3][j][lane]);
}

__global__ __launch_bounds__(256) void k_gemv_cols_finish(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  if (A.scal[blockIdx.y * kScal + kDone] != 0.0) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.np) return;
  const int64_t nch = ceil_div<int64_t>(I.rows, kRowChunk);
  const double* part = A.colpart + I.colpart_off + k;
  double s = 0.0;
  for (int64_t c = 0; c < nch; ++c) s += part[c * I.np];
  const int64_t o = I.param_off + k;
  A.w[o] = A.mask[o] * s / (double)I.rows + A.shift[o] * A.p[o];
}

// alpha = rho / (p . w);  x += alpha p;  r -= alpha w
__global__ void k_cg_xr(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  const double* sc = A.scal + blockIdx.y * kScal;
  if (sc[kDone] != 0.0) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.np) return;
  const double alpha = sc[kRho] / sc[kPw];
  const int64_t o = I.param_off + k;
  A.x[o] += alpha * A.p[o];
  A.r[o] -= alpha * A.w[o];
}

// Convergence test (rho' < eps^2 |b|^2) and beta; one thread per instance.
__global__ void k_cg_check(SrArgs A, int iter) {
  double* sc = A.scal + blockIdx.x * kScal;
  if (sc[kDone] != 0.0) return;
  const double rn = sc[kRhoNew];
  sc[kIters] = (double)iter;
  if (rn < sc[kThresh]) {
    sc[kDone] = 1.0;
    return;
  }
  sc[kBeta] = rn / sc[kRho];
  sc[kRho] = rn;
}

__global__ void k_cg_p(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  const double* sc = A.scal + blockIdx.y * kScal;
  if (sc[kDone] != 0.0) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.np) return;
  const int64_t o = I.param_off + k;
  A.p[o] = A.r[o] + sc[kBeta] * A.p[o];
}

__global__ void k_cg_setup(SrArgs A, double eps) {
  double* sc = A.scal + blockIdx.x * kScal;
  // rho = |r|^2 = |b|^2 is in kRho (k_dot into kRho)
  sc[kThresh] = eps * eps * sc[kRho];
  sc[kDone] = 0.0;
  sc[kIters] = 0.0;
}

// alpha <- alpha - dtau x   (frozen parameters have x = 0)
__global__ void k_apply_update(SrArgs A, double dtau, double* __restrict__ params,
                               double* __restrict__ dparams) {
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= I.np) return;
  const int64_t o = I.param_off + k;
  const double d = -dtau * A.x[o];
  if (dparams) dparams[o] = d;
  params[o] += d;
}

// --------------------------------------------------------------- launchers
void sr_estats(const SrArgs& A, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_estats, dim3(n_inst), dim3(256), 0, s, A);
}

template <typename T>
void sr_colstats(const SrArgs& A, T* O, uint16_t* split, double* g, int n_inst, int64_t max_ld,
                 int64_t max_rows, hipStream_t s) {
  const int cb = (int)ceil_div<int64_t>(max_ld, 256);
  const int ch = (int)ceil_div<int64_t>(max_rows, kRowChunk);
  hipLaunchKernelGGL(k_colpass<T>, dim3(cb, ch, n_inst), dim3(256), 0, s, A, O, 0, split);
  hipLaunchKernelGGL(k_colfinish, dim3(cb, n_inst), dim3(256), 0, s, A, 0, g);
  hipLaunchKernelGGL(k_colpass<T>, dim3(cb, ch, n_inst), dim3(256), 0, s, A, O, 1, split);
  hipLaunchKernelGGL(k_colfinish, dim3(cb, n_inst), dim3(256), 0, s, A, 1, g);
}

template <typename T, typename TS>
void sr_syrk_vec(const SrArgs& A, const T* O, TS* S, int n_inst, int64_t max_np, int max_ksplit,
                 bool any_wide, bool any_narrow, int wide_units, int wide_tail, hipStream_t s) {
  if constexpr (std::is_same<T, double>::value && std::is_same<TS, double>::value) {
    if (any_wide) {
      hipLaunchKernelGGL(k_syrk_f64_wide, dim3(wide_units > 0 ? wide_units : 1, n_inst), dim3(256),
                         0, s, A, O, S);
      if (wide_tail > 0)
        hipLaunchKernelGGL(k_syrk_f64_tail, dim3(kWT * kWT / 256, wide_tail, n_inst), dim3(256), 0,
                           s, A, S);
    }
    if (!any_narrow) return;
  }
  const int nt = (int)ceil_div<int64_t>(max_np, kTile);
  const int ntiles = nt * (nt + 1) / 2;
  if constexpr (std::is_same<T, double>::value)
    hipLaunchKernelGGL(k_syrk_f64mfma, dim3(ntiles, max_ksplit, n_inst), dim3(256), 0, s, A, O);
  else
    hipLaunchKernelGGL(k_syrk_vec<T>, dim3(ntiles, max_ksplit, n_inst), dim3(256), 0, s, A, O);
  hipLaunchKernelGGL(k_syrk_reduce<TS>, dim3(ntiles, kTile * kTile / 256, n_inst), dim3(256), 0, s,
                     A, S);
}

// A trailing update with fewer 128-tiles than this (two workgroups on each of
// 256 compute units, four times over) runs on 64-tiles.  At N_p = 10^4 the
// solve took 15.9, 15.6, 15.2 and 15.5 ms with 512, 1024, 2048 and any
// count (64-tiles throughout).
constexpr int kTrailTiles128 = 2048;

template <typename TS>
void sr_cholesky_solve(const SrArgs& A, const TS* S, const double* g, double eps_rel, double eps_abs,
                       double freeze, int n_inst, int64_t max_np, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_prep<TS>, dim3(max_np, n_inst), dim3(256), 0, s, A, S, g, eps_rel,
                     eps_abs, freeze);
  // two levels: block columns of kNb, left-looking inside outer panels of
  // kOuter (one fused launch per block column, the forward substitution
  // with it), the columns past each outer panel updated once per panel on
  // the matrix cores
  const int nblk = (int)ceil_div<int64_t>(max_np, kNb);
  const int nob = (int)ceil_div<int64_t>(max_np, kOuter);
  constexpr int kPer = kOuter / kNb;
  for (int ob = 0; ob < nob; ++ob) {
    const int kb0 = ob * kPer, kb1 = kb0 + kPer < nblk ? kb0 + kPer : nblk;
    for (int kb = kb0; kb < kb1; ++kb)
      hipLaunchKernelGGL(k_chol_column, dim3(nblk - kb, n_inst), dim3(256), 0, s, A, kb, kb0);
    if (kb1 < nblk) {
      // 128-tiles while they fill the device four times over, then 64-tiles
      const int64_t m = max_np - (int64_t)(ob + 1) * kOuter;
      const int nt128 = (int)ceil_div<int64_t>(m, 128);
      if (nt128 * (nt128 + 1) / 2 >= kTrailTiles128) {
        hipLaunchKernelGGL(k_chol_trail<128>, dim3(nt128 * (nt128 + 1) / 2, n_inst), dim3(256), 0,
                           s, A, ob);
      } else {
        const int nt = (int)ceil_div<int64_t>(m, 64);
        hipLaunchKernelGGL(k_chol_trail<64>, dim3(nt * (nt + 1) / 2, n_inst), dim3(256), 0, s, A,
                           ob);
      }
    }
  }
  // backward substitution: the diagonal blocks inverted at once, then one
  // block row per launch from each instance's own last block
  hipLaunchKernelGGL(k_trtri_diag, dim3(nblk, n_inst), dim3(64), 0, s, A);
  for (int step = 0; step < nblk; ++step) {
    const int b = nblk - 1 - step;   // of the widest instance
    hipLaunchKernelGGL(k_trsv_back, dim3(b > 1 ? b : 1, n_inst), dim3(256), 0, s, A, step);
  }
}

namespace {
void sr_dot(const SrArgs& A, const double* a, const double* b, int slot, int check_done,
            int n_inst, int64_t max_np, hipStream_t s) {
  const int64_t p = ceil_div<int64_t>(max_np, 4096);
  const int parts = (int)(p < kDotParts ? (p > 0 ? p : 1) : kDotParts);
  hipLaunchKernelGGL(k_dot_part, dim3(parts, n_inst), dim3(256), 0, s, A, a, b, check_done);
  hipLaunchKernelGGL(k_dot_finish, dim3(n_inst), dim3(64), 0, s, A, slot, check_done);
}
}  // namespace

template <typename T>
void sr_cg_begin(const SrArgs& A, const double* g, double eps_rel, double eps_abs, double freeze,
                 double eps, int n_inst, int64_t max_np, hipStream_t s) {
  const int cb = (int)ceil_div<int64_t>(max_np, 256);
  hipLaunchKernelGGL(k_cg_init, dim3(cb, n_inst), dim3(256), 0, s, A, g, eps_rel, eps_abs, freeze);
  sr_dot(A, A.r, A.r, kRho, 0, n_inst, max_np, s);
  hipLaunchKernelGGL(k_cg_setup, dim3(n_inst), dim3(1), 0, s, A, eps);
}

template <typename T>
void sr_cg_iter(const SrArgs& A, const T* O, int iter, int n_inst, int64_t max_np, int64_t max_rows,
                hipStream_t s) {
  const int cb = (int)ceil_div<int64_t>(max_np, 256);
  hipLaunchKernelGGL(k_gemv_rows<T>,
                     dim3((unsigned)ceil_div<int64_t>(max_rows, 4 * kRowsPerWave),
                          (unsigned)ceil_div<int64_t>(max_np, kColChunk), n_inst),
                     dim3(256), 0, s, A, O);
  hipLaunchKernelGGL(k_gemv_rows_finish, dim3((unsigned)ceil_div<int64_t>(max_rows, 256), n_inst),
                     dim3(256), 0, s, A);
  hipLaunchKernelGGL(k_gemv_cols_part<T>,
                     dim3((unsigned)ceil_div<int64_t>(max_np, 64 * (16 / (int64_t)sizeof(T))),
                          (unsigned)ceil_div<int64_t>(max_rows, kRowChunk), n_inst),
                     dim3(256), 0, s, A, O);
  hipLaunchKernelGGL(k_gemv_cols_finish, dim3(cb, n_inst), dim3(256), 0, s, A);
  sr_dot(A, A.p, A.w, kPw, 1, n_inst, max_np, s);
  hipLaunchKernelGGL(k_cg_xr, dim3(cb, n_inst), dim3(256), 0, s, A);
  sr_dot(A, A.r, A.r, kRhoNew, 1, n_inst, max_np, s);
  hipLaunchKernelGGL(k_cg_check, dim3(n_inst), dim3(1), 0, s, A, iter);
  hipLaunchKernelGGL(k_cg_p, dim3(cb, n_inst), dim3(256), 0, s, A);
}

void sr_apply(const SrArgs& A, double dtau, double* params, double* dparams, int n_inst,
              int64_t max_np, hipStream_t s) {
  const int cb = (int)ceil_div<int64_t>(max_np, 256);
  hipLaunchKernelGGL(k_apply_update, dim3(cb, n_inst), dim3(256), 0, s, A, dtau, params, dparams);
}

template void sr_colstats<double>(const SrArgs&, double*, uint16_t*, double*, int, int64_t, int64_t,
                                  hipStream_t);
template void sr_colstats<float>(const SrArgs&, float*, uint16_t*, double*, int, int64_t, int64_t,
                                 hipStream_t);
template void sr_syrk_vec<double, double>(const SrArgs&, const double*, double*, int, int64_t, int,
                                          bool, bool, int, int, hipStream_t);
template void sr_syrk_vec<float, float>(const SrArgs&, const float*, float*, int, int64_t, int,
                                        bool, bool, int, int, hipStream_t);
template void sr_cholesky_solve<double>(const SrArgs&, const double*, const double*, double, double,
                                        double, int, int64_t, hipStream_t);
template void sr_cholesky_solve<float>(const SrArgs&, const float*, const double*, double, double,
                                       double, int, int64_t, hipStream_t);
template void sr_cg_begin<double>(const SrArgs&, const double*, double, double, double, double, int,
                                  int64_t, hipStream_t);
template void sr_cg_begin<float>(const SrArgs&, const double*, double, double, double, double, int,
                                 int64_t, hipStream_t);
template void sr_cg_iter<double>(const SrArgs&, const double*, int, int, int64_t, int64_t,
                                 hipStream_t);
template void sr_cg_iter<float>(const SrArgs&, const float*, int, int, int64_t, int64_t, hipStream_t);

}  // namespace mvmc
