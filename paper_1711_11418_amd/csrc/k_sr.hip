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

template <typename TS>
__global__ void k_syrk_reduce(SrArgs A, TS* __restrict__ S) {
  const SrInst& I = A.inst[blockIdx.z];
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

// Cholesky of diagonal block kb, left-looking (Cholesky-Crout), one
// wavefront: lane i keeps row i in registers and finishes it left to right,
//   L[i][j] = (A[i][j] - sum_{m<j} L[i][m] L[j][m]) * (1 / L[j][j]),
//   L[j][j] = sqrt(A[j][j] - sum_{m<j} L[j][m]^2),
// reading the finished row j from LDS.  Entries above the diagonal (and rows
// past the matrix) are computed but never read or stored.  A non-positive
// pivot sets the instance's flag.
__global__ __launch_bounds__(64) void k_potrf_diag(SrArgs A, int kb) {
  const SrInst& I = A.inst[blockIdx.x];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  if (kb >= nblk) return;
  const int64_t o = (int64_t)kb * kNb;
  const int nb = (int)(I.np - o < kNb ? I.np - o : kNb);
  const int i = threadIdx.x;
  if (i >= kNb) return;   // one wavefront per block
  double* F = A.chol + I.chol_off;
  double r[kNb];
  const double* Fi = F + (o + (i < nb ? i : nb - 1)) * I.np + o;
#pragma unroll
  for (int j = 0; j < kNb; ++j) r[j] = Fi[j < nb ? j : nb - 1];
  __shared__ double Ls[kNb][kNb + 1];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    // the dot product in four independent chains (latency, not bandwidth)
    double c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int m = 0; m < j; ++m) c[m & 3] += r[m] * Ls[j][m];
    const double s = r[j] - ((c[0] + c[1]) + (c[2] + c[3]));
    const double dj = lane_value(s, j);
    if (j < nb && !(dj > 0.0)) bad = true;
    const double ljj = sqrt(dj > 0.0 ? dj : DBL_MIN);
    const double rl = 1.0 / ljj;
    r[j] = i == j ? ljj : s * rl;
    Ls[i][j] = r[j];
    wave::wave_sync();
    asm volatile("" ::: "memory");   // keep each row's loads within its step
  }
  if (bad && i == 0) A.scal[blockIdx.x * kScal + kFlag] = 1.0;
  double* Fw = F + (o + i) * I.np + o;
  if (nb == kNb) {
    // whole rows: the part above the diagonal is never read
#pragma unroll
    for (int j = 0; j < kNb; ++j) Fw[j] = r[j];
  } else if (i < nb) {
    for (int j = 0; j <= i; ++j) Fw[j] = Ls[i][j];
  }
}

// Panel below the diagonal block: every row r below it solves
// L[r][blk] L_kk^T = F[r][blk], one thread per row with the row in
// registers and L_kk shared in LDS (256 rows per workgroup).
constexpr int kTrsmRows = 256;
__global__ __launch_bounds__(kTrsmRows) void k_trsm_panel(SrArgs A, int kb) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  if (kb >= nblk) return;
  const int64_t o = (int64_t)kb * kNb;
  const int64_t r0 = o + kNb + (int64_t)blockIdx.x * kTrsmRows;
  if (r0 >= I.np) return;
  const int nb = (int)(I.np - o < kNb ? I.np - o : kNb);
  __shared__ double L[kNb][kNb];
  double* F = A.chol + I.chol_off;
  for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
    const int i = e / kNb, j = e % kNb;
    L[i][j] = (i < nb && j <= i) ? F[(o + i) * I.np + o + j] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  const int64_t row = r0 + threadIdx.x;
  if (row >= I.np) return;
  // columns past the matrix (last block only) read the last column and are
  // replaced by zero, so the loads need no branch
  double x[kNb];
  double* Fr = F + row * I.np;
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    const double v = Fr[o + j < I.np ? o + j : I.np - 1];
    x[j] = j < nb ? v : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kNb; ++j) {
    double s = x[j];
#pragma unroll
    for (int m = 0; m < j; ++m) s -= x[m] * L[j][m];
    x[j] = s / L[j][j];
    asm volatile("" ::: "memory");   // keep each row of L_kk's loads within its step
  }
  if (nb == kNb) {
#pragma unroll
    for (int j = 0; j < kNb; ++j) Fr[o + j] = x[j];
  } else {
    for (int j = 0; j < nb; ++j) {
      double v = x[0];
#pragma unroll
      for (int t = 1; t < kNb; ++t)
        if (t == j) v = x[t];
      Fr[o + j] = v;
    }
  }
}

// Update inside an outer panel: F[ib][jb] -= L[ib][kb] L[jb][kb]^T for the
// later blocks jb of the panel (kb < jb < jb_end) and every block row
// ib >= jb (lower triangle).  The columns past the panel are left to
// k_chol_trail, which applies the whole panel at once.
__global__ __launch_bounds__(256) void k_chol_update(SrArgs A, int kb, int jb_end) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  const int jend = jb_end < nblk ? jb_end : nblk;
  int idx = blockIdx.x, jb = kb + 1;
  while (jb < jend && idx >= nblk - jb) {
    idx -= nblk - jb;
    ++jb;
  }
  if (jb >= jend) return;
  const int ib = jb + idx;
  const int64_t o = (int64_t)kb * kNb, ro = (int64_t)ib * kNb, co = (int64_t)jb * kNb;
  const int nk = (int)(I.np - o < kNb ? I.np - o : kNb);
  const int nr = (int)(I.np - ro < kNb ? I.np - ro : kNb);
  const int nc = (int)(I.np - co < kNb ? I.np - co : kNb);
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double Ms[kNb][kNb + 1];
  double* F = A.chol + I.chol_off;
  for (int e = threadIdx.x; e < kNb * kNb; e += blockDim.x) {
    const int i = e / kNb, k = e % kNb;
    Ls[i][k] = (i < nr && k < nk) ? F[(ro + i) * I.np + o + k] : 0.0;
    Ms[i][k] = (i < nc && k < nk) ? F[(co + i) * I.np + o + k] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int k = 0; k < nk; ++k) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = Ls[ty * 4 + i][k];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Ms[tx * 4 + j][k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty * 4 + i, c = tx * 4 + j;
      if (r < nr && c < nc && (ib != jb || c <= r)) F[(ro + r) * I.np + co + c] -= acc[i][j];
    }
}

// Trailing update of outer step ob: the lower triangle of the rows and
// columns past the outer panel [o, o + kOuter) less L[:, panel] L[:, panel]^T,
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  A workgroup of four
// wavefronts owns a 128 x 128 tile, each wavefront a 64 x 64 quadrant as
// 4 x 4 blocks of 16 x 16 accumulators.  The panel's columns pass through
// LDS k-major (each MFMA operand is 16 consecutive doubles of one column),
// 16 at a time, double-buffered; rows past the matrix read the last row.
// Two workgroups share a compute unit (two wavefronts per SIMD), which the
// FP64 matrix unit needs to stay busy.
constexpr int kOuter = 4 * kNb;   // outer panel width
constexpr int kUT = 128;          // trailing-update tile
constexpr int kUK = 16;           // panel columns per LDS stage
constexpr int kUP = kUT + 2;      // padded LDS row (spreads the four k rows of an operand over the banks)
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256, 2) void k_chol_trail(SrArgs A, int ob) {
  const SrInst& I = A.inst[blockIdx.y];
  const int64_t o = (int64_t)ob * kOuter, t0 = o + kOuter;
  if (t0 >= I.np) return;
  const int nt = (int)ceil_div<int64_t>(I.np - t0, kUT);
  if ((int)blockIdx.x >= nt * (nt + 1) / 2) return;
  int ti = 0, start = 0;   // lower-triangle tile (ti >= tj)
  while ((int)blockIdx.x >= start + ti + 1) {
    start += ti + 1;
    ++ti;
  }
  const int tj = (int)blockIdx.x - start;
  const int64_t r0 = t0 + (int64_t)ti * kUT, c0 = t0 + (int64_t)tj * kUT;
  double* F = A.chol + I.chol_off;
  __shared__ double As[2][kUK][kUP];
  __shared__ double Bs[2][kUK][kUP];
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int qi = wv >> 1, qj = wv & 1;
  const int lr = tid >> 1, lk = (tid & 1) * (kUK / 2);   // staging: half a stage row of row lr
  const int64_t ra = r0 + lr, rb = c0 + lr;
  const double* pa = F + (ra < I.np ? ra : I.np - 1) * I.np + o + lk;
  const double* pb = F + (rb < I.np ? rb : I.np - 1) * I.np + o + lk;
  double ga[kUK / 2], gb[kUK / 2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < kUK / 2; ++e) {
      ga[e] = pa[k0 + e];
      gb[e] = pb[k0 + e];
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int e = 0; e < kUK / 2; ++e) {
      As[st][lk + e][lr] = ga[e];
      Bs[st][lk + e][lr] = gb[e];
    }
  };
  f64x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  gload(0);
  lstore(0);
  __syncthreads();
  int st = 0;
  const int ka = lane >> 4, ma = lane & 15;   // operand element: k row, row within the block
  for (int k0 = 0; k0 < kOuter; k0 += kUK) {
    const bool more = k0 + kUK < kOuter;
    if (more) gload(k0 + kUK);
#pragma unroll
    for (int kk = 0; kk < kUK; kk += 4) {
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
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 64 * qi + 16 * i + ka + 4 * r;
        const int64_t col = c0 + 64 * qj + 16 * j + ma;
        if (row < I.np && col < I.np && (ti != tj || col <= row)) F[row * I.np + col] -= acc[i][j][r];
      }
}

// Inverse of every 64 x 64 diagonal block of the factor, all blocks at once
// (one wavefront each), stored row-major after the factor at
// chol_off + np^2 + kb * 64^2.  Lane j forms column j by forward
// substitution, L z = e_j:  z_i = (delta_ij - sum_{m<i} L[i][m] z_m) / L[i][i],
// with L_kk in LDS and the columns in LDS.  Rows and columns past the matrix
// (last block) are the identity.
__global__ __launch_bounds__(64) void k_trtri_diag(SrArgs A) {
  const SrInst& I = A.inst[blockIdx.y];
  const int kb = blockIdx.x;
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  if (kb >= nblk) return;
  const int64_t o = (int64_t)kb * kNb;
  const int nb = (int)(I.np - o < kNb ? I.np - o : kNb);
  const double* F = A.chol + I.chol_off;
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double Zs[kNb][kNb + 1];
  const int j = threadIdx.x;
  for (int i = 0; i < kNb; ++i) {
    Ls[i][j] = (i < nb && j <= i) ? F[(o + i) * I.np + o + j] : (i == j ? 1.0 : 0.0);
    Zs[i][j] = 0.0;
  }
  wave::wave_sync();
  for (int i = 0; i < kNb; ++i) {
    double s = i == j ? 1.0 : 0.0;
    for (int m = j; m < i; ++m) s -= Ls[i][m] * Zs[m][j];
    Zs[i][j] = i < j ? 0.0 : s / Ls[i][i];
  }
  wave::wave_sync();
  double* Li = A.chol + I.chol_off + I.np * I.np + (int64_t)kb * kNb * kNb;
  for (int i = 0; i < kNb; ++i) Li[i * kNb + j] = Zs[i][j];
}

// Substitution in groups of G diagonal blocks, in place in x: group gi is
// blocks kb0, kb0 + 1, ... with kb0 = G gi (forward) or kb0, kb0 - 1, ...
// with kb0 = nblk - 1 - G gi (backward, from each instance's own last block).
// One workgroup per instance solves the group: for each block b of it, with
// the blocks of the group before it already solved,
//   forward   x_b <- Linv_bb (x_b - sum L[b][c] x_c)          (c earlier in the group)
//   backward  x_b <- Linv_bb^T (x_b - sum L[c][b]^T x_c)      (c later in the group)
// every 64 x 64 block staged through LDS by all threads at once (sixteen
// loads in flight per thread), then one thread per row (forward) or column
// (backward) of the 64.  Contributions of blocks outside the group come from
// k_trsv_rest.
constexpr int kTrsvG = 8;
__global__ __launch_bounds__(256) void k_trsv_group(SrArgs A, int gi, int transpose) {
  const SrInst& I = A.inst[blockIdx.x];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  const int kb0 = transpose ? nblk - 1 - gi * kTrsvG : gi * kTrsvG;   // first block of group gi
  if (kb0 >= nblk || kb0 < 0) return;
  const double* F = A.chol + I.chol_off;
  const double* Lv = F + I.np * I.np;
  double* x = A.x + I.param_off;
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double xs[kTrsvG][kNb];   // solved blocks of the group
  __shared__ double xb[kNb];
  const int tid = threadIdx.x;
  // stage a 64 x 64 block (rows r0.., columns c0.., nr x nc valid) into Ls
  auto stage = [&](const double* src, int64_t ld, int nr, int nc) {
    double v[kNb * kNb / 256];
#pragma unroll
    for (int u = 0; u < kNb * kNb / 256; ++u) {
      const int e = tid + 256 * u, i = e / kNb, m = e % kNb;
      v[u] = (i < nr && m < nc) ? src[(int64_t)i * ld + m] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kNb * kNb / 256; ++u) {
      const int e = tid + 256 * u;
      Ls[e / kNb][e % kNb] = v[u];
    }
  };
  for (int g = 0; g < kTrsvG; ++g) {
    const int b = transpose ? kb0 - g : kb0 + g;
    if (b < 0 || b >= nblk) break;   // uniform
    const int64_t ob = (int64_t)b * kNb;
    const int nb = (int)(I.np - ob < kNb ? I.np - ob : kNb);
    if (tid < kNb) xb[tid] = tid < nb ? x[ob + tid] : 0.0;
    // contributions of the blocks of the group solved before b
    for (int g2 = 0; g2 < g; ++g2) {
      const int c = transpose ? kb0 - g2 : kb0 + g2;
      const int64_t oc = (int64_t)c * kNb;
      const int nc = (int)(I.np - oc < kNb ? I.np - oc : kNb);
      __syncthreads();   // Ls free, xb written
      if (!transpose) stage(F + ob * I.np + oc, I.np, nb, nc);   // L[b][c]
      else stage(F + oc * I.np + ob, I.np, nc, nb);              // L[c][b]
      __syncthreads();
      if (tid < kNb) {
        double s = 0.0;
        if (!transpose)
          for (int m = 0; m < kNb; ++m) s += Ls[tid][m] * xs[g2][m];
        else
          for (int i = 0; i < kNb; ++i) s += Ls[i][tid] * xs[g2][i];
        xb[tid] -= s;
      }
    }
    __syncthreads();
    stage(Lv + (int64_t)b * kNb * kNb, kNb, kNb, kNb);
    __syncthreads();
    if (tid < kNb) {
      double y = 0.0;
      if (!transpose)
        for (int m = 0; m < kNb; ++m) y += Ls[tid][m] * xb[m];
      else
        for (int i = 0; i < kNb; ++i) y += Ls[i][tid] * xb[i];
      xs[g][tid] = y;
      if (tid < nb) x[ob + tid] = y;
    }
  }
}

// The solved group's contribution to every block outside it: one workgroup
// per target block t (forward: t after the group; backward: t before it),
//   forward   x_t -= sum over the group's blocks c of L[t][c] x_c
//   backward  x_t -= sum over the group's blocks c of L[c][t]^T x_c
// Forward: a wavefront per 16 rows of t, lanes across the group's columns,
// the 16 rows' loads of a column chunk in flight together, one wave sum per
// row.  Backward: lanes across the 64 columns of t, the four wavefronts
// splitting the group's rows (eight loads in flight), partial sums added in
// wavefront order.
__global__ __launch_bounds__(256) void k_trsv_rest(SrArgs A, int gi, int transpose) {
  const SrInst& I = A.inst[blockIdx.y];
  const int nblk = (int)ceil_div<int64_t>(I.np, kNb);
  const int kb0 = transpose ? nblk - 1 - gi * kTrsvG : gi * kTrsvG;
  if (kb0 >= nblk || kb0 < 0) return;
  // group blocks [c0, c1)
  const int c0 = transpose ? (kb0 - kTrsvG + 1 > 0 ? kb0 - kTrsvG + 1 : 0) : kb0;
  const int c1 = transpose ? kb0 + 1 : (kb0 + kTrsvG < nblk ? kb0 + kTrsvG : nblk);
  const int t = transpose ? (int)blockIdx.x : c1 + (int)blockIdx.x;
  if (transpose ? t >= c0 : t >= nblk) return;
  const double* F = A.chol + I.chol_off;
  double* x = A.x + I.param_off;
  const int64_t ot = (int64_t)t * kNb, gc0 = (int64_t)c0 * kNb;
  const int64_t gc1 = ((int64_t)c1 * kNb < I.np ? (int64_t)c1 * kNb : I.np);
  const int nt = (int)(I.np - ot < kNb ? I.np - ot : kNb);
  const int ncols = (int)(gc1 - gc0);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double xg[kTrsvG * kNb];
  __shared__ double part[4][kNb];
  for (int e = tid; e < ncols; e += 256) xg[e] = x[gc0 + e];
  __syncthreads();
  if (!transpose) {
    constexpr int RW = kNb / 4;   // rows per wavefront
    double acc[RW];
#pragma unroll
    for (int u = 0; u < RW; ++u) acc[u] = 0.0;
    for (int m0 = 0; m0 < ncols; m0 += 64) {
      const int m = m0 + lane;
      const double xm = m < ncols ? xg[m] : 0.0;
#pragma unroll
      for (int u = 0; u < RW; ++u) {
        const int i = wv + 4 * u;
        acc[u] += (i < nt && m < ncols) ? F[(ot + i) * I.np + gc0 + m] * xm : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const int i = wv + 4 * u;
      const double v = wave::wave_total(acc[u]);
      if (lane == 0 && i < nt) x[ot + i] -= v;
    }
  } else {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (lane < nt)
      for (int i0 = wv * 8; i0 < ncols; i0 += 32) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          a[u] += i < ncols ? F[(gc0 + i) * I.np + ot + lane] * xg[i] : 0.0;
        }
      }
    part[wv][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (tid < nt) x[ot + tid] -= ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
  }
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
#pragma unroll 4
  for (int64_t k = c0 + lane; k < c1; k += 64) {
    const double pk = p[k] * mk[k];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r)
      if (r < nr) s[r] += (double)row[r * I.ldO + k] * pk;
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
  const SrInst& I = A.inst[blockIdx.z];
  if (A.scal[blockIdx.z * kScal + kDone] != 0.0) return;
  const int64_t m0 = (int64_t)blockIdx.y * kRowChunk;
  if (m0 >= I.rows) return;
  const int64_t m1 = m0 + kRowChunk < I.rows ? m0 + kRowChunk : I.rows;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * 64 + lane;
  const double* t = A.t + I.eloc_off;
  double s = 0.0;
  if (k < I.np) {
    const T* col = O + I.O_off + k;
#pragma unroll 8
    for (int64_t m = m0 + wv; m < m1; m += 4) s += (double)col[m * I.ldO] * t[m];
  }
  __shared__ double red[4][64];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && k < I.np)
    A.colpart[I.colpart_off + (int64_t)blockIdx.y * I.np + k] =
        (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
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
                 hipStream_t s) {
  const int nt = (int)ceil_div<int64_t>(max_np, kTile);
  const int ntiles = nt * (nt + 1) / 2;
  if constexpr (std::is_same<T, double>::value)
    hipLaunchKernelGGL(k_syrk_f64mfma, dim3(ntiles, max_ksplit, n_inst), dim3(256), 0, s, A, O);
  else
    hipLaunchKernelGGL(k_syrk_vec<T>, dim3(ntiles, max_ksplit, n_inst), dim3(256), 0, s, A, O);
  hipLaunchKernelGGL(k_syrk_reduce<TS>, dim3(ntiles, kTile * kTile / 256, n_inst), dim3(256), 0, s,
                     A, S);
}

template <typename TS>
void sr_cholesky_solve(const SrArgs& A, const TS* S, const double* g, double eps_rel, double eps_abs,
                       double freeze, int n_inst, int64_t max_np, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_prep<TS>, dim3(max_np, n_inst), dim3(256), 0, s, A, S, g, eps_rel,
                     eps_abs, freeze);
  // two levels: blocks of kNb factored inside outer panels of kOuter, the
  // columns past each outer panel updated once per panel on the matrix cores
  const int nblk = (int)ceil_div<int64_t>(max_np, kNb);
  const int nob = (int)ceil_div<int64_t>(max_np, kOuter);
  constexpr int kPer = kOuter / kNb;
  for (int ob = 0; ob < nob; ++ob) {
    const int kb0 = ob * kPer, kb1 = kb0 + kPer < nblk ? kb0 + kPer : nblk;
    for (int kb = kb0; kb < kb1; ++kb) {
      hipLaunchKernelGGL(k_potrf_diag, dim3(n_inst), dim3(kNb), 0, s, A, kb);
      const int R = nblk - kb - 1;
      if (R > 0) {
        const int rows = (int)(max_np - (int64_t)(kb + 1) * kNb);
        hipLaunchKernelGGL(k_trsm_panel, dim3(ceil_div(rows, kTrsmRows), n_inst), dim3(kTrsmRows),
                           0, s, A, kb);
        int tiles = 0;
        for (int jb = kb + 1; jb < kb1; ++jb) tiles += nblk - jb;
        if (tiles)
          hipLaunchKernelGGL(k_chol_update, dim3(tiles, n_inst), dim3(256), 0, s, A, kb, kb1);
      }
    }
    if (kb1 < nblk) {
      const int nt = (int)ceil_div<int64_t>(max_np - (int64_t)(ob + 1) * kOuter, kUT);
      hipLaunchKernelGGL(k_chol_trail, dim3(nt * (nt + 1) / 2, n_inst), dim3(256), 0, s, A, ob);
    }
  }
  // substitutions: the diagonal blocks inverted at once, then groups of
  // kTrsvG blocks, each solved by one workgroup and applied to the blocks
  // outside it (group gi counts from the first block forward and from each
  // instance's own last block backward)
  hipLaunchKernelGGL(k_trtri_diag, dim3(nblk, n_inst), dim3(64), 0, s, A);
  const int ngrp = ceil_div(nblk, kTrsvG);
  for (int t = 0; t < 2; ++t)
    for (int gi = 0; gi < ngrp; ++gi) {
      hipLaunchKernelGGL(k_trsv_group, dim3(n_inst), dim3(256), 0, s, A, gi, t);
      const int rest = nblk - (gi + 1) * kTrsvG;   // most target blocks of any instance
      if (rest > 0)
        hipLaunchKernelGGL(k_trsv_rest, dim3(rest, n_inst), dim3(256), 0, s, A, gi, t);
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
                     dim3((unsigned)ceil_div<int64_t>(max_np, 64),
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
                                          hipStream_t);
template void sr_syrk_vec<float, float>(const SrArgs&, const float*, float*, int, int64_t, int,
                                        hipStream_t);
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
